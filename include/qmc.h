/*
 * qmc.h -- C ABI of libqmc, an MI355X (gfx950) implementation of one population-dynamics time
 * step of the real-time, sign-problem-suppressed quantum Monte Carlo of Shen & Lidar,
 * arXiv:2502.18929.
 *
 * The problem (eq. (1)): d rho/dt = -i[H(t), rho] + (1/2) sum_k gamma_k(t) D[L_k] rho with
 * D[L] rho = 2 L rho L^dagger - {L^dagger L, rho}.  The density matrix is column-stacked
 * (eq. (2)) and represented per replica by an integer population vector |N(t)> of complex
 * walkers (eq. (3) and the End Matter on spawn and annihilation).
 *
 * Conventions
 *  - Qubit q of the basis state |i> is bit q of i.  The element |i><j| (ket i, bra j) has the
 *    walker key (j << n) | i (2n bits).
 *  - A monomial (x, z, re, im) is the operator (re + i im) X^x Z^z with
 *    X^x Z^z |i> = (-1)^popcount(z & i) |i ^ x>.  x and z use the low n bits.
 *  - A population is a Gaussian integer (re, im) of int32 walker counts (signs +-1, +-i).
 *
 * Arithmetic contract (identical in the CPU oracle that checks this library bit for bit)
 *  - Every source term of the Liouvillian (kappa0 * A rho B for Pauli monomials A, B) is scaled
 *    per step by its weight w (s_m(t_s) for H monomial m, gamma_k(t_s) for L_k) and quantized
 *    as q = llrint(ldexp(dt * (w * kappa0), 32)) separately for Re and Im; equal (target mask,
 *    sign mask) pairs are then merged by integer addition.  A column group (all terms with the
 *    same key-XOR mask) must satisfy sum(|q_re| + |q_im|) < 2^31, else QMC_ERR_DT.
 *  - Per parent (key, a + ib) and step s, Philox4x32-10 with key (seed_lo, seed_hi) and counter
 *    (key_lo32, key_hi32, s, replica << 8) yields words w0 (spawn) and w1 (death).
 *  - Death/cloning: the diagonal coefficient d(key) times (a + ib), both components rounded
 *    with one systematic comb started at w1, added to N(t).  Spawning: the off-diagonal groups
 *    in increasing mask order, Re then Im of each, rounded with one comb started at w0; nonzero
 *    children go to key ^ mask.  A comb over Q32 values x_k with start U emits
 *    sign(x_k) * floor((r_k + |x_k|) / 2^32), r_0 = U, r_{k+1} = (r_k + |x_k|) mod 2^32, whose
 *    expectation is exactly x_k / 2^32 (the unbiasedness identity of the End Matter).
 *  - Annihilation: parents and children are summed per key in int64; a sum outside int32 is
 *    QMC_ERR_COUNT_OVERFLOW; (0, 0) locations disappear.
 *
 * Memory and threading
 *  - The caller owns every host array passed in (copied during the call) and every output
 *    array (written during the call).
 *  - The caller owns the device workspace (any device allocation, e.g. a torch uint8 tensor of
 *    qmc_workspace_bytes bytes) and the HIP stream; all device work of a context is enqueued
 *    on that stream.  The library never allocates device memory; it allocates pinned host
 *    staging memory in qmc_init and frees it in qmc_destroy.
 *  - One context per stream; calls on one context must not overlap.
 *
 * Errors: every int-returning function returns QMC_OK (0) or a negative code; no exception
 * crosses the ABI.  After an error qmc_last_error gives a message.  Device-side errors are
 * detected at the end of each qmc_step batch; the context then holds the last good step
 * (the step before the one that failed), so a caller may re-initialize with more capacity,
 * qmc_import that state and repeat the step with an identical result.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define QMC_OK 0
#define QMC_ERR_ARG (-1)            /* invalid argument (sizes, masks, ordering, capacity) */
#define QMC_ERR_DT (-2)             /* a column group violates the Q32 bound; nothing ran */
#define QMC_ERR_STORE_CAP (-3)      /* more occupied keys than the store capacity */
#define QMC_ERR_SPAWN_CAP (-4)      /* more child records in one step than the spawn capacity */
#define QMC_ERR_COUNT_OVERFLOW (-5) /* an annihilated population left the int32 range */
#define QMC_ERR_HIP (-6)            /* a HIP runtime call failed (no device, launch failure) */
#define QMC_ERR_STATE (-8)          /* the context is unusable after an earlier HIP error */

typedef struct { uint64_t x, z; double re, im; } qmc_monomial;

typedef struct {
  uint32_t n_qubits;        /* 1..32, and 2*n_qubits + ceil(log2(n_replicas)) <= 64 */
  uint32_t n_replicas;      /* independent samples of eq. (3), all advanced together */
  uint64_t seed;            /* Philox key */
  double dt;                /* Euler time step (End Matter on simulation methodology) */
  uint64_t walker_target;   /* N^diag of the eq. (3) paragraph; only used for reporting */
  uint64_t store_capacity;  /* occupied keys per replica the store can hold */
  uint64_t spawn_capacity;  /* child records per replica per step */
  /* Population control (FCIQMC background paragraph; the update rule of Booth, Thom & Alavi,
   * J. Chem. Phys. 131, 054106 (2009)).  shift_mode 0 (default): the shift of each replica is
   * the constant of qmc_set_shift (0 unless set; the paper needs none, the Liouvillian being
   * trace preserving).  shift_mode 1: after every step whose index is a multiple of
   * shift_period (A >= 1), a replica whose N^tot has reached shift_target takes its N^tot as
   * the reference (the first time) or updates its shift, S <- S - shift_zeta / (A dt) *
   * ln(N^tot(s) / N^tot(s - A)) (FP64, natural logarithm; an empty replica keeps S).  The shift
   * adds to the death coefficient (L_diag + S) and biases the estimators.  Euler only. */
  uint32_t shift_mode;
  double shift_zeta;        /* damping zeta >= 0 */
  uint32_t shift_period;    /* A */
  uint64_t shift_target;    /* N^tot at which a replica's shift starts to vary */
} qmc_config;

/* H(t) = sum_m s_m(t) h[m] with real weights s_m(t) given per step; L_k = sum of the monomials
 * l[l_off[k]] .. l[l_off[k+1]-1] with real rates gamma_k(t) given per step (negative rates are
 * allowed: the time-local, non-Markovian case of eq. (1)).  l_off has n_l + 1 entries. */
typedef struct {
  uint32_t n_h;
  const qmc_monomial* h;
  uint32_t n_l;
  const uint32_t* l_off;
  const qmc_monomial* l;
} qmc_model;

typedef struct qmc_ctx qmc_ctx;

/* Bytes of device workspace a context with this configuration needs: the population vectors
 * N(t) of eq. (3) for every replica (16 bytes per occupied key of the column-stacked density
 * matrix of eq. (2), store_capacity keys per replica, in two buffers), one step's child records
 * (spawn_capacity per replica) and the per-step working areas.  QMC_ERR_ARG on an invalid
 * configuration. */
int qmc_workspace_bytes(const qmc_config* cfg, const qmc_model* model, size_t* bytes);

/* Create a context (eq. (3) paragraph: N(0) := N^diag rho(0)).  keys/re/im are the n0 initial
 * records of every replica: keys < 2^(2n) sorted ascending and unique, no (0, 0) population.
 * d_workspace is a device pointer to ws_bytes >= qmc_workspace_bytes bytes, 256-byte aligned,
 * owned by the caller and kept alive until qmc_destroy.  hip_stream is a hipStream_t (NULL =
 * the default stream).  Errors: QMC_ERR_ARG, QMC_ERR_HIP. */
int qmc_init(const qmc_config* cfg, const qmc_model* model, const uint64_t* keys,
             const int32_t* re, const int32_t* im, uint64_t n0, void* d_workspace,
             size_t ws_bytes, void* hip_stream, qmc_ctx** out);

/* A batch of circuits in one context (the spec batched step): n_circuits models on the
 * same n qubits (a smaller circuit leaves the extra qubits idle: its masks and keys use only its
 * own qubits), each with its own initial records (keys[c], re[c], im[c], n0[c], as qmc_init)
 * and cfg->n_replicas replicas.  Replica r of circuit c is store segment s = c * n_replicas + r:
 * its composite key is (s << 2n) | key, its Philox stream id is s, and every call that takes a
 * replica index (qmc_export, qmc_import, qmc_set_shift, qmc_observe's output rows) takes s.
 * Capacities are per segment.  qmc_step takes the weights of all circuits side by side:
 * s[nsteps][sum_c n_h(c)], gamma[nsteps][sum_c n_l(c)], circuit c's after those of circuits
 * 0..c-1.  One step advances every circuit with its own table; on the fused path every key
 * range holds one circuit's keys.  The AB2 integrator and the initiator approximation run one
 * circuit per context (QMC_ERR_ARG otherwise).  1 <= n_circuits <= 512 and at most the number
 * of co-resident workgroups of the fused step (256 on MI355X); QMC_ERR_ARG otherwise. */
int qmc_workspace_bytes_batch(const qmc_config* cfg, uint32_t n_circuits,
                              const qmc_model* models, size_t* bytes);
int qmc_init_batch(const qmc_config* cfg, uint32_t n_circuits, const qmc_model* models,
                   const uint64_t* const* keys, const int32_t* const* re,
                   const int32_t* const* im, const uint64_t* n0, void* d_workspace,
                   size_t ws_bytes, void* hip_stream, qmc_ctx** out);

/* Advance every replica by nsteps Euler steps (End Matter, spawn and annihilation steps,
 * Euler solver).  s is [nsteps][n_h] and gamma is [nsteps][n_l], row k holding the weights at
 * the left end t = (step0 + k) * dt of step k.  Tables are quantized and bound-checked on the
 * host before the call changes any state (QMC_ERR_DT or QMC_ERR_ARG for a table leaves the state
 * untouched; the LDS-resident step may start its first batch into scratch segments while the
 * later tables are checked, and a failing table cancels it); device errors
 * (QMC_ERR_STORE_CAP, QMC_ERR_SPAWN_CAP, QMC_ERR_COUNT_OVERFLOW) roll the context back to the
 * last good step.  Synchronizes the stream once at the end. */
int qmc_step(qmc_ctx* ctx, uint32_t nsteps, const double* s, const double* gamma);

/* Which implementation qmc_step launches; every choice gives the same result bit for bit.
 * path 0 (default): automatic -- the fused persistent kernel (one launch per batch of steps,
 * one grid barrier per step, every key range owned by one workgroup) while the store holds at
 * most 8192 keys per co-resident workgroup and no key range overflows its segment or its
 * per-step inbox, otherwise the streamed kernels (spawn, radix sort of the children, merge)
 * for the next 256 steps; and before both, while every replica (store segment) has at most
 * qmc_small_limit occupied keys, the Euler step with the comb runs LDS-resident: one workgroup
 * per segment holds it and takes batches of up to 64 steps with no grid-wide synchronization
 * (a segment that outgrows the limit, or whose step would need more than 1024 records on
 * unoccupied keys or exceed a capacity, hands the step over to the fused kernel for the rest of
 * the trajectory, until the next qmc_import, qmc_step_path or qmc_small_limit).  path 1: fused
 * only (an overflowing key range is reported as QMC_ERR_STORE_CAP or QMC_ERR_SPAWN_CAP).
 * path 2: streamed only.  path 3: LDS-resident only, up to 1024 keys per segment
 * (QMC_ERR_STORE_CAP when a segment does not fit; QMC_ERR_ARG with AB2, a spawn proposal, step
 * tables above 8 KB or more segments than co-resident workgroups).  QMC_ERR_ARG otherwise. */
int qmc_step_path(qmc_ctx* ctx, int32_t path);

/* Keys per replica up to which the automatic path takes the LDS-resident step (default 384;
 * 0 = never; at most QMC_SMALL_MAX_KEYS, else QMC_ERR_ARG).  One workgroup then carries a whole
 * replica, so the limit trades the fused kernel's per-step grid synchronization against the
 * work of one workgroup; it changes no result. */
#define QMC_SMALL_MAX_KEYS 1024
int qmc_small_limit(qmc_ctx* ctx, uint32_t keys);

/* Time integrator of qmc_step (End Matter on simulation methodology): 0 = Euler (default),
 * N(s+1) = N(s) + round(dt L(t_s) N(s)); 1 = AB2, for s >= 1
 *   N(s+1) = N(s) + round(3/2 dt L(t_s) N(s)) + round(-1/2 dt L(t_{s-1}) N(s-1)),
 * each term rounded as in the Euler step from its own table -- Q32 of scale * (dt * (w * kappa))
 * with scale 3/2 and -1/2 -- and its own Philox stream (0 for N(s), 1 for N(s-1), whose diagonal
 * is a record of its own rather than a change of N(s-1)).  Refused (QMC_ERR_ARG) with the
 * variable shift.  The context keeps N(s-1) and the
 * weights of step s-1; without them (after qmc_init, qmc_set_integrator or qmc_pulse) the next
 * step is an Euler step.  Switching clears N(s-1).  QMC_ERR_ARG for another value.  An AB2
 * step whose two tables have more than 257 column groups between them is refused by qmc_step
 * with QMC_ERR_ARG (a key's records from both tables must stay within one merge run). */
int qmc_set_integrator(qmc_ctx* ctx, int32_t integrator);

/* AB2: N(s-1) of one replica (same record rules as qmc_init) and the weights of step s-1
 * (s_prev[n_h], gamma_prev[n_l], shared by all replicas), for a context resumed at step s
 * (qmc_import) with the next step an AB2 step.  A replica whose N(s-1) is not set has an empty
 * one.  QMC_ERR_ARG if the integrator is not AB2 or the records are invalid. */
int qmc_set_prev(qmc_ctx* ctx, uint32_t replica, const uint64_t* keys, const int32_t* re,
                 const int32_t* im, uint64_t n, const double* s_prev, const double* gamma_prev);

/* AB2: copy one replica's N(s-1) to host arrays, as qmc_export.  QMC_ERR_ARG if there is none. */
int qmc_export_prev(qmc_ctx* ctx, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
                    uint64_t cap, uint64_t* n);

/* Ideal instantaneous Pauli pulse on every replica: rho -> P rho P^dagger with P = X^x Z^z,
 * i.e. |i><j| -> (-1)^{popc(z & i) + popc(z & j)} |i ^ x><j ^ x| (used for the staggered-XX
 * dynamical-decoupling pulses of Fig. 1(c)).  With AB2 the next step is an Euler step. */
int qmc_pulse(qmc_ctx* ctx, uint64_t x, uint64_t z);
/* The same for a batch: circuit c takes P = X^x[c] Z^z[c] (arrays of n_circuits entries). */
int qmc_pulse_batch(qmc_ctx* ctx, const uint64_t* x, const uint64_t* z);

/* Diagonal shift S of one replica (death coefficient L_diag + S): the constant value, or the
 * current value of a variable shift (shift_mode 1), which later updates start from.  The paper
 * needs none (the Liouvillian is trace preserving); S != 0 biases the estimator. */
int qmc_set_shift(qmc_ctx* ctx, uint32_t replica, double shift);

/* Initiator approximation (End Matter on simulation methodology, last paragraph): from the next
 * step on, a parent whose population |re| + |im| is below min_walkers (the caller's
 * xi * N^diag rounded up to whole walkers) is not an initiator, and every record it spawns onto
 * a key that is not occupied in N(s) is discarded; death on its own key always counts.  With
 * AB2 the second term's parents are judged by their population in N(s-1), their targets
 * against N(s).  0 turns it off (the default: the plain step).  The rule is applied where the
 * records are merged: a routed record's key carries one flag bit below the composite key.
 * Errors: QMC_ERR_ARG when 2n + replica bits leave no bit for the flag (2n + bits > 63). */
int qmc_set_initiator(qmc_ctx* ctx, uint64_t min_walkers);

/* Spawn proposal (End Matter, spawn step: the multinomial over a column's (target, Re/Im)
 * channels, with importance weights so the expectation stays dt L N).  kind 0 = the plain comb
 * over every channel (default); otherwise each parent draws `samples` channels (a power of two,
 * 1..64) with fixed-point probabilities P_ch / 2^32 and puts round(x_ch / (samples P_ch)) walkers
 * on each, x_ch being the channel's Q32 amount, rounded exactly from the offset of the uniform
 * inside the channel's interval.  P_ch: a floor of 2^32 / (16 nch) each, the rest in proportion to
 * weights W_ch -- kind 1 uniform (W = 1), kind 2 heat-bath (|x_ch| scaled below 2^24), kind 3 the
 * scores of an int8 MLP of the key bits: input b = +1 / -1 where bit b of the key (2n bits) is
 * set / clear, 0 up to 64; hidden h_j = min(127, max(0, b1[j] + w1[j] . input) >> hidden_shift),
 * 32 units; score_g = b2[g-1] + w2[g-1] . h for groups g = 1..64 (W = min(2^24, max(0, score))
 * for both components, 0 past 64).  w1 int8 [32][64], b1 int32 [32], w2 int8 [64][32], b2 int32
 * [64], row-major host arrays, copied (kind 3 only; NULL otherwise).  Death keeps its comb.
 * Sample k of a parent draws Philox stream 0x40 + k.  Runs on the streamed path (the automatic
 * path switches to it; a fused-only context refuses the step).  Errors: QMC_ERR_ARG for a bad
 * kind, sample count or shift, with AB2, the initiator approximation or several circuits, and
 * at qmc_step when samples x (column groups - 1) + 1 exceeds 256 for a step's table;
 * QMC_ERR_COUNT_OVERFLOW when one drawn record exceeds the int32 range. */
int qmc_set_proposal(qmc_ctx* ctx, int32_t kind, uint32_t samples, const int8_t* w1,
                     const int32_t* b1, const int8_t* w2, const int32_t* b2,
                     uint32_t hidden_shift);

/* Spawn proposal kind 4, the learned proposal's deeper network (End Matter, spawn step, as
 * above; the learned-proposal configuration's inputs): channel weights W of both components of
 * group g = min(2^24, max(0, score_{g-1})), 0 past 64 groups, from an int8 network with 128
 * inputs -- +1 / -1 where key bit b is set / clear for b < 2n, then one input per weight channel
 * of the step (the model's H monomials, then its Lindblad operators), 1 where that channel's
 * weight is nonzero at the step and 0 where it is zero, 0 past -- two hidden layers of 128 units,
 * h1 = min(127, max(0, b1 + w1 . x) >> shift1), h2 = min(127, max(0, b2 + w2 . h1) >> shift2), and
 * score_g = b3[g] + w3[g] . h2.  w1 int8 [128][128], b1 int32 [128], w2 int8 [128][128],
 * b2 int32 [128], w3 int8 [64][128], b3 int32 [64]: row-major host arrays, copied.  The hidden
 * layers run as int8 MFMA products with int32 accumulation.  `samples` as above; the same
 * refusals as qmc_set_proposal (QMC_ERR_ARG), and shifts above 30.  qmc_set_proposal(kind 0)
 * switches it off. */
int qmc_set_proposal_deep(qmc_ctx* ctx, uint32_t samples, const int8_t* w1, const int32_t* b1,
                          const int8_t* w2, const int32_t* b2, const int8_t* w3,
                          const int32_t* b3, uint32_t shift1, uint32_t shift2);

/* Spawn-event log, the training data of a learned proposal (the learned-proposal configuration:
 * spawn events of the plain method).  From the next qmc_step on, every nonzero off-diagonal child
 * that the streamed path draws with the plain comb (End Matter, spawn step) is appended to
 * d_events as 24 bytes {uint64 parent composite key (segment << 2n | key), uint32 step, uint32
 * column group g >= 1 of that step's table, int32 re, int32 im} (device memory, caller-owned)
 * while fewer than `capacity` are stored; *d_count (device uint64, caller-owned, set by the
 * caller) counts every event, so a count above capacity means events were dropped.  Events of
 * one step come in no particular order.  The fused and LDS-resident paths and proposals log
 * nothing: use qmc_step_path(ctx, 2) while logging.  d_events = NULL switches it off.
 * QMC_ERR_ARG when d_events is given without d_count. */
int qmc_log_spawns(qmc_ctx* ctx, void* d_events, uint64_t capacity, uint64_t* d_count);

/* Tile size of the look-back radix sort, which re-sorts the whole store after a pulse with x
 * flips (records per thread of a 256-thread tile: 8, 12, 16 or 24; 16 by default; the sort of
 * each streamed step's records uses tiles of 2048 and no look-back, whatever this is set to).
 * The digit width is 11 bits in both.  records_per_thread = 0 autotunes: every size
 * is timed three times on synthetic records of this context's composite-key width and spawn
 * capacity (at most 4M records) in the child buffers, and the fastest is kept; nonzero sets it.
 * The sorted order, and so every result, is the same for every size.  *chosen (may be NULL)
 * receives the size in use.  Call between steps (the child buffers are scratch then).  Errors:
 * QMC_ERR_ARG for an unsupported size; QMC_ERR_HIP if a timing run fails (the context is then
 * unusable). */
int qmc_tune_sort(qmc_ctx* ctx, uint32_t records_per_thread, uint32_t* chosen);

/* Streamed chunks as HIP graphs: with on = 1 every chunk of streamed steps (spawn, and per step
 * the sort passes, merge split points and merge) is captured from the context's stream into a
 * graph; the executable graph of the previous chunk is updated with it when the launches are
 * the same (only arguments changed), else a new one is instantiated; then it is launched.  The
 * results are identical; profiling (qmc_profile) runs the chunks eagerly.  Default 0. */
int qmc_use_graphs(qmc_ctx* ctx, int32_t on);

typedef struct {
  uint32_t n_pauli;          /* observables P = X^px Z^pz: sum_i (-1)^popc(pz&i) N_{i,i^px} */
  const uint64_t* px;
  const uint64_t* pz;
  uint32_t n_psi;            /* sparse |psi> for the fidelity <psi|rho|psi> (Fig. 2 caption) */
  const uint64_t* psi_index;
  const double* psi_re;
  const double* psi_im;
  uint32_t want_eps;         /* nonzero: anti-Hermiticity numerator (End Matter) */
} qmc_obs_spec;

/* Outputs, arrays of length n_replicas (times the per-replica counts shown), caller-owned.
 * Integer numerators are exact.  FP64 values are normalized by N^diag(0) of that replica
 * (eq. (3)): trace = Re N^diag(t) / Re N^diag(0) (replica-aggregation paragraph), theta =
 * atan2(Im N^diag, Re N^diag) (End Matter on sign-problem suppression), pauli_val = numerator
 * / Re N^diag(0), fidelity = Re sum_{u,v} conj(psi_u) psi_v N_{uv} / Re N^diag(0) with N_{uv}
 * at key (v << n) | u, eps = sqrt(sum |N_ij - conj N_ji|^2) / Re N^diag(0). */
typedef struct {
  uint64_t* n_occ;           /* [R] occupied keys (dim H_QMC of the scaling paragraph) */
  uint64_t* n_tot;           /* [R] sum |re| + |im| (N^tot) */
  int64_t* ndiag;            /* [R][2] */
  int64_t* pauli;            /* [R][n_pauli][2] */
  uint64_t* eps2;            /* [R][2] 128-bit (lo, hi) */
  double* trace;             /* [R] */
  double* theta;             /* [R] */
  double* pauli_val;         /* [R][n_pauli][2] */
  double* fidelity;          /* [R][2] (Re, Im) */
  double* eps;               /* [R] */
  double* shift;             /* [R] the shift S now: nonzero means biased estimators (not
                                written by qmc_observe_noalloc, which has no context) */
} qmc_obs_out;

/* Estimators of the current state (any NULL output pointer is skipped). */
int qmc_observe(qmc_ctx* ctx, const qmc_obs_spec* spec, qmc_obs_out* out);

/* For callers that cannot allocate (code under HIP graph capture, tight serving loops, harnesses
 * that forbid allocation): the estimators of qmc_observe on a store the caller holds in device
 * memory, with no context and no allocation of any kind.  d_keys are n composite keys
 * (replica << 2 n_qubits) | key, sorted ascending and unique, and d_vals the n (re, im) int32
 * pairs beside them (2n int32), both device pointers owned by the caller (a context's store, or
 * any copy of one); nd0_re is a host array of Re N^diag(0) per replica, which normalizes the FP64
 * outputs (it may be NULL when no FP64 output is asked for).  spec and out are as for
 * qmc_observe, with the same values.  Every scratch word -- staged inputs, accumulators,
 * lookups, outputs before their copy back -- lives in one device array of
 * QMC_NOALLOC_SCRATCH_BYTES bytes inside the library, one per device, held until the process
 * ends; its address is taken on the first call on each device.  Each GPU has one such array
 * which every call on it shares: calls that overlap on one GPU race, so callers on one GPU must
 * serialize them (the array keeps the last call's contents; each call clears what it
 * accumulates).  Limits: n_replicas <= QMC_NOALLOC_MAX_REPLICAS, n_pauli <=
 * QMC_NOALLOC_MAX_PAULI, n_psi <= QMC_NOALLOC_MAX_PSI and n_psi^2 x n_replicas <=
 * QMC_NOALLOC_MAX_LOOKUPS; beyond them QMC_ERR_ARG, as for a mask outside n bits or a missing
 * pointer.  Enqueued on hip_stream (NULL = the default stream), which is synchronized before the
 * call returns.  QMC_ERR_HIP if a launch or copy fails. */
#define QMC_NOALLOC_MAX_REPLICAS 256
#define QMC_NOALLOC_MAX_PAULI 64
#define QMC_NOALLOC_MAX_PSI 32
#define QMC_NOALLOC_MAX_LOOKUPS 32768
#define QMC_NOALLOC_SCRATCH_BYTES 1359104
int qmc_observe_noalloc(uint32_t n_qubits, uint32_t n_replicas, const uint64_t* d_keys,
                        const int32_t* d_vals, uint64_t n, const int64_t* nd0_re,
                        const qmc_obs_spec* spec, qmc_obs_out* out, void* hip_stream);

/* Copy one replica's store -- its population vector N(t) of eq. (3), the occupied keys of the
 * column-stacked density matrix of eq. (2) with their Gaussian-integer walker counts -- to host
 * arrays (keys ascending).  *n receives the size; if it exceeds cap nothing is copied and
 * QMC_ERR_ARG is returned. */
int qmc_export(qmc_ctx* ctx, uint32_t replica, uint64_t* keys, int32_t* re, int32_t* im,
               uint64_t cap, uint64_t* n);

/* Replace one replica's store (its population vector N(t) of eq. (3); same rules as qmc_init's
 * records) and set the step counter of the context to `step` (the Philox counter of the next
 * step: the draws are keyed on the walkers, so (store, step) is the whole state of a replica).  N(s-1) (AB2) is left as it
 * is; qmc_set_prev replaces it. */
int qmc_import(qmc_ctx* ctx, uint32_t replica, const uint64_t* keys, const int32_t* re,
               const int32_t* im, uint64_t n, uint32_t step);

/* Counters of a context: the step counter, the occupied keys of all replicas now, and running
 * sums since qmc_init over the parents of every step of N^tot (walker_steps), occupied keys
 * (key_steps), routed records (child_steps: the nonzero death/cloning deltas, which travel as
 * records of the parent's own key, and the children), annihilated output keys (out_steps) and
 * off-diagonal children alone (spawn_steps, the spawned walkers' records of the End Matter spawn
 * step).  The sums give the walker-steps/s and key-steps/s rates and the algorithmic bytes of
 * the kernels.
 * `rebalances` counts the times the fused kernel re-cut its key ranges to even out a grown
 * population, inside one launch or by stopping for a new one (no effect on the results). */
typedef struct {
  uint32_t step;
  uint64_t n_occ_total;
  uint64_t walker_steps;
  uint64_t key_steps;
  uint64_t child_steps;
  uint64_t out_steps;
  uint64_t rebalances;
  uint64_t spawn_steps;
} qmc_stats;

int qmc_counters(qmc_ctx* ctx, qmc_stats* out);

/* Live timing of one kernel class with HIP events recorded on the context's stream around
 * every launch of that class in qmc_step: kernel_class 0 = streamed draws (the records of each
 * step from its parents: death/cloning and children), 1 = streamed record sort (all radix
 * passes), 2 = streamed annihilation (tile split points, tile output counts and offsets, and the
 * merge), 3 = one launch of the fused persistent kernel (a batch of whole steps), 4 = one
 * launch of the LDS-resident step (a batch of whole steps), 5 = one chunk of whole streamed
 * steps (from the chunk's first draws to its last merge: draws, sorts and merges of every step,
 * End Matter spawn and annihilation steps), -1 = off.
 * qmc_profile resets the totals.  qmc_profile_read returns the summed milliseconds, the number of
 * timed launches and, in `covered` (may be NULL), the counter sums (walker_steps, key_steps,
 * child_steps, out_steps, spawn_steps, and in `step` the number of steps) of exactly the steps
 * that the timed launches ran -- for classes 1 to 4; zeros for class 0.  The algorithmic
 * bytes of the timed kernels follow from these sums.  The two whole-step classes are timed
 * together: with class 3 or 4 selected, launches of both are timed, each into its own totals,
 * which qmc_profile_read_class returns for any class (zeros for a class not timed); class 5
 * also times class 2 into its own totals; QMC_ERR_ARG for a class outside 0..5. */
int qmc_profile(qmc_ctx* ctx, int32_t kernel_class);
int qmc_profile_read(qmc_ctx* ctx, double* ms, uint64_t* launches, qmc_stats* covered);
int qmc_profile_read_class(qmc_ctx* ctx, int32_t kernel_class, double* ms, uint64_t* launches,
                           qmc_stats* covered);

/* The quantized coefficient table of one step for this configuration and model, computed on
 * the host only (no device, no context), for scale * dt * L(t) (scale 1 for Euler, 3/2 and -1/2
 * for the two AB2 terms): n_groups groups (group 0 = diagonal, always present)
 * with masks gxmask[g] and term ranges gstart[g] .. gstart[g+1]-1; term t has sign mask
 * tzmask[t] and Q32 coefficient tq[t][0] + i tq[t][1].  For checking the table against an
 * independent implementation.  QMC_ERR_ARG if a capacity is too small, QMC_ERR_DT if the
 * Q32 bound fails. */
int qmc_coeff_table(const qmc_config* cfg, const qmc_model* model, const double* s,
                    const double* gamma, double scale, uint32_t cap_groups, uint32_t cap_terms,
                    uint32_t* n_groups, uint64_t* gxmask, uint32_t* gstart, uint32_t* n_terms,
                    uint64_t* tzmask, int64_t* tq);

/* Message of the last error on this context (owned by the context, valid until its next
 * call), or a static string when ctx is NULL. */
const char* qmc_last_error(const qmc_ctx* ctx);

void qmc_destroy(qmc_ctx* ctx);

#ifdef __cplusplus
}
#endif
#endif
