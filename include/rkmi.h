/*
 * rkmi.h -- C ABI of the MI355X batched ODE integrators.
 *
 * Integrates very many independent ODE systems dy/dt = f(t, y, g), each with
 * its own initial state y(t0) and constant parameters g, from t0 to t1
 * (Niemeyer & Sung 2014, Sec. 2, Eq. 1), by
 *   - RKCK: adaptive fifth-order Runge-Kutta-Cash-Karp (Sec. 2.1, Table 1,
 *     driver of Sec. 3.1), for nonstiff systems;
 *   - RKC: adaptive second-order Runge-Kutta-Chebyshev (Sec. 2.2, driver of
 *     Sec. 3.2, nonlinear power method of the Appendix), for moderately stiff
 *     systems.
 * Every call restarts the integrator (Sec. 3: no step-size memory between
 * calls), as an operator-split caller needs.
 *
 * Conventions for every entry point:
 *   - Arrays are FP64 (states, parameters) or int32 (status, statistics),
 *     struct-of-arrays: element (row r, system i) sits at [r * n_sys + i], so
 *     the same unknown of consecutive systems is contiguous (Sec. 3).
 *   - Array arguments are DEVICE pointers on the current HIP device, owned by
 *     the caller, 8-byte aligned (4 for int32).  The library checks that each
 *     is device memory but cannot check its extent: the caller guarantees the
 *     sizes stated per argument.
 *   - Work is enqueued on `stream` (a hipStream_t; NULL = the null stream) and
 *     the call returns without waiting.  Outputs are valid once the stream has
 *     reached that point.
 *   - Return value: RK_OK, or a negative RK_E* code when the arguments are
 *     rejected or the launch fails; then nothing was enqueued (launch failures
 *     excepted) and rk_last_error() describes the problem.
 *   - Numerical failure of a single system is not an error of the call: it
 *     is reported in that system's `status` entry; its output is the last
 *     accepted state and the other systems are unaffected.
 */
#ifndef RKMI_H
#define RKMI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Return codes. */
#define RK_OK 0
#define RK_EINVAL (-1)        /* invalid argument */
#define RK_ENOMEM (-2)        /* host or device allocation failed */
#define RK_EHIP (-3)          /* HIP runtime or launch error */
#define RK_EUNSUPPORTED (-4)  /* no compiled code for this problem / method */
#define RK_EWORKSPACE (-5)    /* workspace missing or too small */

/* Per-system status. */
#define RK_SYS_OK 0
#define RK_SYS_NONFINITE 1    /* an accepted state was not finite */
#define RK_SYS_HMIN 2         /* step fell below the minimum after a rejection */
#define RK_SYS_MAXSTEPS 3     /* max_steps attempts used before reaching t1 */
#define RK_SYS_TAPE 4         /* adjoint: the tape or workspace could not hold the system's
                                 steps or stages; its gradients are NaN */

/* Rows of the per-system statistics array. */
#define RK_STAT_ACCEPT 0      /* accepted steps */
#define RK_STAT_REJECT 1      /* rejected attempts */
#define RK_STAT_RHS 2         /* right-hand-side evaluations */
#define RK_STAT_SR_CALLS 3    /* spectral-radius estimates (RKC) */
#define RK_STAT_POW_ITERS 4   /* power-method iterations (RKC) */
#define RK_STAT_MAX_STAGES 5  /* largest stage count used (RKC; 6 for RKCK) */
#define RK_NSTATS 6

typedef struct rk_problem_s *rk_problem;

/* A reversible mass-action network (host arrays, copied by the library).
 * Rate law, isothermal at constant volume (Sec. 4.2 species equations):
 *   C_k = rho Y_k / W_k,  [M] = sum_k C_k,
 *   k_f,j = exp(lnA_j + beta_j ln T - Ea_j / T),   k_r,j = k_f,j / Keq_j
 *   (Sec. 4.2 Arrhenius form, Ea in kelvin, i.e. E/R),
 *   q_j = k_f,j prod_{reactant slots} C - k_r,j prod_{product slots} C,
 *         where a side with a single species is multiplied by [M],
 *   dY_k/dt = (W_k / rho) sum_j nu_kj q_j.
 * reac/prod: [n_rx][2] species indices in [0, n_sp), second slot -1 for a
 * one-species side.  Per-system parameters g = (T, rho): rows 0 and 1. */
typedef struct {
  int32_t n_sp;
  int32_t n_rx;
  const int32_t *reac;
  const int32_t *prod;
  const double *lnA;    /* [n_rx] */
  const double *beta;   /* [n_rx] */
  const double *Ea;     /* [n_rx] kelvin */
  const double *Keq;    /* [n_rx] > 0 */
  const double *W;      /* [n_sp] > 0 */
} rk_mech_desc;

/* Options; pass NULL for the defaults of the paper's listings. */
typedef struct {
  int64_t max_steps;    /* attempts per system before RK_SYS_MAXSTEPS; <= 0: 10^7 */
  int32_t sr_period;    /* RKC: spectral radius every this many accepted steps; <= 0: 25 */
  int32_t sr_itmax;     /* RKC: power-method iteration limit; <= 0: 50 */
  int32_t schedule;     /* RK_SCHED_*: 0 automatic (persistent when the workspace is large
                           enough, else plain), 1 plain, 2 persistent (needs workspace) */
  int32_t refill;       /* persistent schedule: a wave takes new systems once at least this
                           many of its 64 lanes are idle (1..64; <= 0: tuned default) */
  int32_t cost_order;   /* nonzero: hand systems to lanes in decreasing order of their cost,
                           estimated by a pilot integration at loosened tolerances (see
                           RK_SCHED_* below); results are unchanged.  Taped
                           integrations work in the tape's own order area; not for
                           batches (RK_EUNSUPPORTED). */
  int32_t sr_method;    /* RKC spectral radius: 0 the nonlinear power method (Appendix),
                           1 the Gershgorin bound max_k sum_i |J_ki| of the analytic
                           Jacobian (the Appendix's circle-theorem alternative; van der Pol
                           and the isothermal networks of up to 16 species, RK_EUNSUPPORTED
                           otherwise and for taped integrations and batches); unused by
                           RKCK */
  int32_t group_align;  /* group schedule, RKC: a group whose next step is its error
                           estimate and controller waits while another group of its wave is
                           at most this many evaluations from its own, so that the wave runs
                           that code once for both (results are unchanged); 0: the default
                           (1; no waiting with the energy equation), < 0: never wait.
                           Unused by RKCK, whose groups run whole attempts in step. */
  int32_t reserved[3];  /* set to 0 */
} rk_options;

/* Library version (major * 10000 + minor * 100 + patch). */
int rk_version(void);

/* Message describing the last failed call on this host thread ("" if none). */
const char *rk_last_error(void);

/* Van der Pol oscillators (Sec. 2 Eq. 1 with N = 2): f = (y2, mu (1 - y1^2) y2 - y1);
 * one parameter per system, g row 0 = mu.  *out receives a handle to release
 * with rk_problem_destroy. */
int rk_problem_create_vdp(rk_problem *out);

/* The Pleiades problem (Sec. 4.1): seven bodies of mass m_i = i in the plane,
 * 28 unknowns per system in the order x_1..x_7, y_1..y_7, x_1'..x_7',
 * y_1'..y_7'; f = (velocities, accelerations) with
 *   x_i'' = sum_{j != i} m_j (x_j - x_i) / r_ij,  y_i'' likewise,
 *   r_ij = ((x_i - x_j)^2 + (y_i - y_j)^2)^(3/2),
 * the 3/2 power formed as d2 sqrt(d2) and the division as a multiplication by
 * the pair's reciprocal.  No per-system parameters (pass g = NULL).  The
 * group schedule (the default, RK_SCHED_AUTO) spreads a system over eight
 * lanes with its vectors in registers; the plain and persistent schedules run
 * one lane per system with its vectors in workspace columns.  Every schedule
 * needs rk_workspace_bytes (the group one for its queue).  All schedules give
 * the same bits.  No adjoint (RK_EUNSUPPORTED). */
int rk_problem_create_pleiades(rk_problem *out);

/* Mass-action network described by *desc (host memory, copied).  The network
 * topology must have been compiled into the library (see the package's code
 * generator); RK_EUNSUPPORTED otherwise. */
int rk_problem_create_mass_action(const rk_mech_desc *desc, rk_problem *out);

/* The network of *desc with the energy equation of Sec. 4.2 at constant
 * volume (adiabatic): state (T, Y_1..Y_N), N + 1 unknowns, row 0 = T in
 * kelvin; one parameter per system, g row 0 = rho (constant);
 *   dY_k/dt = W_k omega_k / rho  (omega_k as rk_problem_create_mass_action,
 *             with k_f,j = exp(lnA_j + beta_j ln T - Ea_j / T) at the current T),
 *   dT/dt   = -(sum_k e_k omega_k W_k) / (rho c_v),  c_v = sum_k Y_k c_v,k(T),
 *   e_k(T)  = u0_k + (cv0_k + cv1_k T) T,  c_v,k(T) = cv0_k + 2 cv1_k T
 * (per unit mass; u0, cv0, cv1: host arrays of n_sp, copied).  Available for
 * the topologies the code generator was given with the energy equation
 * (RK_EUNSUPPORTED otherwise): up to 15 species on the one-lane kernels of
 * every schedule; above, the group kernels (32 lanes per system) run under
 * every schedule and need the queue workspace of rk_workspace_bytes.  No
 * adjoint. */
int rk_problem_create_mass_action_thermal(const rk_mech_desc *desc, const double *u0,
                                          const double *cv0, const double *cv1,
                                          rk_problem *out);

/* Releases a problem handle and its device copies (NULL is ignored).  No
 * integration using it may still be pending on any stream. */
void rk_problem_destroy(rk_problem p);

/* Unknowns per system, parameters per system (rows of g), and differentiable
 * parameters (mass action: n_rx, the ln A_j; van der Pol: 1, mu). */
int rk_problem_dims(rk_problem p, int32_t *n_eq, int32_t *n_param, int32_t *n_theta);

/* Schedules.  Plain: one lane per system, system i on global lane i (the
 * paper's intDriver, Sec. 3).  Persistent: a machine-sized grid whose lanes take
 * the next system from a device-side queue as soon as theirs is finished.
 * Group: for networks of more than 16 species, 16 lanes (up to 32 species)
 * or 32 lanes (more species) of a wave share one
 * system (its vectors and rate constants spread over their registers, its
 * concentrations and rates exchanged through LDS), groups taking systems
 * from the queue; other problems run their default.  Auto: group where
 * available, else persistent (plain without a workspace).
 *
 * Cost order (rk_options.cost_order, with any schedule): the lanes of a wave
 * run in lockstep, so a wave lasts as long as its most expensive system.  The
 * call first integrates every system at rtol and atol multiplied by 10^5
 * (rtol at most 1e-3, never below the call's own) for at most 128 attempts,
 * keeping only each system's count of attempted steps, sorts the systems by that count on the
 * device, and then integrates them at the requested tolerances handed out in
 * decreasing order of it.  Each system's result is bit-for-bit the same as
 * without the order.  The workspace grows by 24 + 4 bytes per system plus
 * 33 KiB. */
#define RK_SCHED_AUTO 0
#define RK_SCHED_PLAIN 1
#define RK_SCHED_PERSISTENT 2
#define RK_SCHED_GROUP 3

#define RK_METHOD_RKCK 0
#define RK_METHOD_RKC 1

/* Device workspace (bytes) an integration of n_sys systems by `method` needs
 * under *opt (NULL = defaults) on the current device.  Layout: a 256-byte
 * queue head, then per-workgroup blocks of per-lane columns.  Systems of up to
 * 16 unknowns keep their vectors in registers: 0 bytes for the plain schedule,
 * the queue head for the persistent one.  Larger systems keep every vector and
 * their rate constants in the workspace: one block per 64 systems for the
 * plain schedule, one per resident workgroup for the persistent one (a smaller
 * workspace, down to one block, runs a smaller persistent grid).  RK_SCHED_AUTO
 * sizes for the persistent schedule.  With cost_order the order's buffers
 * follow (256-byte aligned).  Returns 0 on a NULL handle or bad method.  The caller allocates it; it must not be shared by calls that may
 * run concurrently. */
size_t rk_workspace_bytes(rk_problem p, int32_t method, int64_t n_sys, const rk_options *opt);

/* RKCK integration of n_sys systems from t0 to t1 (Sec. 2.1, Sec. 3.1):
 *   y0     [N][n_sys]  initial states
 *   y1     [N][n_sys]  final states (may equal y0: in place)
 *   g      [P][n_sys]  per-system parameters (P from rk_problem_dims)
 *   t0, t1 with t1 >= t0 (t1 == t0 copies y0 to y1)
 *   rtol   > 0: the eps of the paper's error scale;  atol >= 0 enters as
 *          delta = atol / rtol, so a component's allowed error is
 *          rtol (|y| + |h f|) + atol
 *   status [n_sys] or NULL, stats [RK_NSTATS][n_sys] or NULL
 *   ws, ws_bytes: workspace of at least rk_workspace_bytes(...) bytes */
int rk_integrate_rkck(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                      const double *g, double t0, double t1, double rtol, double atol,
                      int32_t *status, int32_t *stats, void *ws, size_t ws_bytes,
                      const rk_options *opt, void *stream);

/* RKC integration (Sec. 2.2, Sec. 3.2, Appendix); arguments as for RKCK, with
 * the weighted RMS error norm of Eq. E:rmsE: weights atol + rtol max(|y_n|, |y_{n+1}|). */
int rk_integrate_rkc(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                     const double *g, double t0, double t1, double rtol, double atol,
                     int32_t *status, int32_t *stats, void *ws, size_t ws_bytes,
                     const rk_options *opt, void *stream);

/* RKC integration as rk_integrate_rkc that allocates nothing, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation).  Its workspace is the library's
 * own device array of RK_SCRATCH_BYTES bytes on each GPU (held from the
 * library's load until the process ends); a call whose workspace would be
 * larger (rk_workspace_bytes with the same arguments) returns RK_EWORKSPACE
 * and enqueues nothing.  Every call on a GPU shares that GPU's array: calls
 * that overlap on one GPU (several streams or host threads at once) race, so
 * serialize them; each call starts from its own cleared queue and order
 * counters, whatever the previous call left.  The problem's constants must
 * already be on the current device: the first allocating call with the
 * problem on that device (any other rk_integrate_* call with n_sys > 0 and
 * t1 > t0) puts them there; otherwise RK_EINVAL.  Other arguments, layouts,
 * ownership and errors as rk_integrate_rkc. */
#define RK_SCRATCH_BYTES (64u << 20)
int rk_integrate_rkc_noalloc(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                             const double *g, double t0, double t1, double rtol, double atol,
                             int32_t *status, int32_t *stats, const rk_options *opt,
                             void *stream);

/* Controller state carried from one call to the next instead of the restart
 * at every call (Sec. 3 notes that carrying the integrator's data across
 * global steps may perform better where the application allows it).  carry:
 * device [rk_carry_rows(p)][n_sys] doubles, caller-owned, read and rewritten
 * by the call; rows
 *   0 valid (0: restart this system, as rk_integrate_*; a call leaves 1 when
 *     the system ended RK_SYS_OK, else 0), 1 the next step size (the one the
 *     controller wanted before the final step was cut to t1), 2 the previous
 *     step, 3 the previous error, 4 the spectral radius, 5 the accepted-step
 *     count that schedules its refresh every 25 steps, 6 whether a previous
 *     step exists, 7..7+N-1 the power method's eigenvector estimate;
 * RKCK uses rows 0 and 1.  y0 and f(t0, y0) are always this call's (the
 * caller may have changed the state between calls).  Zero the array before
 * the first call.  Other arguments as rk_integrate_rkck / rk_integrate_rkc
 * (the cost order's pilot leaves the carried state alone). */
size_t rk_carry_rows(rk_problem p);
int rk_integrate_rkck_carry(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                            const double *g, double t0, double t1, double rtol, double atol,
                            int32_t *status, int32_t *stats, double *carry, void *ws,
                            size_t ws_bytes, const rk_options *opt, void *stream);
int rk_integrate_rkc_carry(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                           const double *g, double t0, double t1, double rtol, double atol,
                           int32_t *status, int32_t *stats, double *carry, void *ws,
                           size_t ws_bytes, const rk_options *opt, void *stream);

/* ---------------------------------------------------------------------------
 * Discrete adjoints of RKC (Sec. 2.2 stage recursion, transposed) and of RKCK
 * (Sec. 2.1 stage equations with the Table 1 coefficients, transposed).
 *
 * The gradient is that of the map y(t0), theta -> y(t1) through the accepted
 * steps, with every step size h_k (and, for RKC, stage count s_k) held at the
 * values the controller chose; the controller, the spectral-radius estimates
 * and the rejected attempts are not differentiated.  theta: the ln A_j of a
 * mass-action network (both rate constants of reaction j scale with A_j), or
 * mu for van der Pol.  Available for systems of up to 16 unknowns
 * (RK_EUNSUPPORTED otherwise).
 *
 * A forward call records a tape (device memory the caller allocates): per
 * system the accepted-step count, each accepted step's (h, s) (s = 6 for
 * RKCK), and the state every ckpt_every accepted steps.  Layout, for n = n_sys, C = max_accepted,
 * K = ckpt_every, each system's records contiguous:
 *   int32 count[n]          (-1: more than C accepted steps; no gradient)
 *   double h[n][Hs], int32 s[n][Hs]   (step k of system i at [i][k])
 *   double y[n][Cs]                   (checkpoint c of system i at [i][c N .. c N + N - 1])
 *   the cost order's working area (seven int32 per system and 32 KiB)
 * with Hs = C and Cs = (C / K + 1) N, each rounded up to a multiple of 16, and
 * each array starting on a 256-byte boundary.  The reverse call recomputes
 * each segment of K steps from its checkpoint and each step's stages, and
 * carries lambda = dL/dy(t1) back to dL/dy(t0).  The same n_sys, g,
 * max_accepted and ckpt_every must be passed to both calls.
 * ------------------------------------------------------------------------- */

/* Bytes of a tape for n_sys systems of at most max_accepted accepted steps,
 * with a checkpoint every ckpt_every accepted steps (0 on bad arguments). */
size_t rk_tape_bytes(rk_problem p, int64_t n_sys, int64_t max_accepted, int32_t ckpt_every);

/* RKC integration as rk_integrate_rkc (one lane per system), recording the
 * tape.  tape: device memory of at least rk_tape_bytes(...) bytes, 256-byte
 * aligned.  A system with more accepted steps than max_accepted integrates
 * normally but its tape count is -1. */
int rk_integrate_rkc_taped(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                           const double *g, double t0, double t1, double rtol, double atol,
                           int32_t *status, int32_t *stats, void *tape, size_t tape_bytes,
                           int64_t max_accepted, int32_t ckpt_every, const rk_options *opt,
                           void *stream);

/* RKCK integration as rk_integrate_rkck (one lane per system), recording the
 * tape as rk_integrate_rkc_taped does. */
int rk_integrate_rkck_taped(rk_problem p, int64_t n_sys, const double *y0, double *y1,
                            const double *g, double t0, double t1, double rtol, double atol,
                            int32_t *status, int32_t *stats, void *tape, size_t tape_bytes,
                            int64_t max_accepted, int32_t ckpt_every, const rk_options *opt,
                            void *stream);

/* Workspace bytes of rk_adjoint_rkc: per system max_stages stage records of
 * N + 4 doubles and ckpt_every states, then the order in which the sweep hands
 * systems to lanes (decreasing accepted steps, from the tape: seven int32 per
 * system and 32 KiB; results do not depend on it) (0 on bad arguments).
 * max_stages bounds the recorded stage counts (RK_STAT_MAX_STAGES of the
 * forward call). */
size_t rk_adjoint_workspace_bytes(rk_problem p, int64_t n_sys, int32_t max_stages,
                                  int32_t ckpt_every);

/* Reverse sweep over a tape from rk_integrate_rkc_taped:
 *   dL_dy1    [N][n_sys]        lambda at t1 (for L = sum w . y(t1): w)
 *   dL_dy0    [N][n_sys]        out: dL/dy(t0)
 *   dL_dtheta [n_theta][n_sys]  out (or NULL): per-system dL/dtheta; for the
 *                               network's shared ln A, sum over systems
 *   status    [n_sys] or NULL   out: RK_SYS_OK, or RK_SYS_TAPE (NaN gradients)
 *   ws, ws_bytes: at least rk_adjoint_workspace_bytes(...) bytes.
 * Asynchronous on `stream`; argument errors are returned before anything is
 * enqueued. */
int rk_adjoint_rkc(rk_problem p, int64_t n_sys, const double *g, const void *tape,
                   size_t tape_bytes, int64_t max_accepted, int32_t ckpt_every,
                   int32_t max_stages, const double *dL_dy1, double *dL_dy0,
                   double *dL_dtheta, int32_t *status, void *ws, size_t ws_bytes,
                   void *stream);

/* Workspace bytes of rk_adjoint_rkck: per system 12 N doubles (the six stage
 * arguments and their adjoints) and ckpt_every states, then the sweep's order
 * as for rk_adjoint_rkc (0 on bad arguments). */
size_t rk_adjoint_rkck_workspace_bytes(rk_problem p, int64_t n_sys, int32_t ckpt_every);

/* Reverse sweep over a tape from rk_integrate_rkck_taped; arguments as for
 * rk_adjoint_rkc (no stage bound), ws of at least
 * rk_adjoint_rkck_workspace_bytes(...) bytes. */
int rk_adjoint_rkck(rk_problem p, int64_t n_sys, const double *g, const void *tape,
                    size_t tape_bytes, int64_t max_accepted, int32_t ckpt_every,
                    const double *dL_dy1, double *dL_dy0, double *dL_dtheta, int32_t *status,
                    void *ws, size_t ws_bytes, void *stream);

/* ---------------------------------------------------------------------------
 * Ragged batches: the systems of several compiled networks of different sizes
 * (each network's systems in their own [N][n] block), integrated with RKC over
 * operator-splitting substeps [t0 + k dt, t0 + (k + 1) dt], k < n_substeps,
 * each substep a restart (Sec. 3), the state updated in place.
 *
 * RK_BATCH_PERSISTENT: one persistent launch per substep for all networks.
 *   Every wave takes the networks in `order` and drains each network's
 *   device queue in turn; lanes freed by finished systems take the next ones
 *   (refill threshold per network), so a wave's live lanes stay packed and
 *   one code path runs per wave.
 * RK_BATCH_PLAIN_INTERLEAVED: one plain launch per substep over n_total
 *   interleaved slots; slot i integrates system (slot_map[i] & 0x0fffffff) of
 *   problem slot_map[i] >> 28, each lane running its own network's code.
 * RK_BATCH_PLAIN_PER_NETWORK: one plain launch per network per substep.
 * use_graph: the substeps are captured once into a HIP graph, replayed while
 *   the call's arguments are unchanged.
 * ------------------------------------------------------------------------- */
typedef struct rk_batch_s *rk_batch;

#define RK_BATCH_PERSISTENT 0
#define RK_BATCH_PLAIN_INTERLEAVED 1
#define RK_BATCH_PLAIN_PER_NETWORK 2

typedef struct {
  int32_t mode;          /* RK_BATCH_* */
  int32_t waves_per_cu;  /* persistent grid: workgroups per compute unit; 0 = occupancy limit */
  int32_t order[4];      /* persistent: problem indices in the order waves take them;
                            order[0] < 0 = largest networks first */
  int32_t refill[4];     /* persistent: idle lanes that trigger a refill, per problem; 0 = 16 */
  int32_t use_graph;     /* nonzero: capture the substeps in one HIP graph */
  int32_t reserved[4];   /* must be zero */
} rk_batch_schedule;

/* A batch over n_prob (1..4) network problems, given in the order every array
 * argument of the batch calls follows.  The set of topologies must have been
 * compiled into the library as a batch (RK_EUNSUPPORTED otherwise). */
int rk_batch_create(const rk_problem *probs, int32_t n_prob, rk_batch *out);

/* Releases the batch and its captured graph (not its problems).  No call using
 * it may still be pending. */
void rk_batch_destroy(rk_batch b);

/* Device workspace bytes of rk_batch_integrate_rkc for n_sys[k] systems per
 * problem (n_total: their sum, used by the interleaved form) under *sched
 * (NULL = persistent, defaults) on the current device; 0 on bad arguments. */
size_t rk_batch_workspace_bytes(rk_batch b, const int64_t *n_sys, int64_t n_total,
                                const rk_batch_schedule *sched);

/* Integrates every system of the batch over n_substeps substeps of dt from t0.
 *   n_sys[k]            systems of problem k
 *   y[k]                [N_k][n_sys[k]] device, updated in place
 *   g[k]                [2][n_sys[k]] device (T, rho)
 *   status[k], stats[k] device [n_sys[k]] / [RK_NSTATS][n_sys[k]], or a NULL
 *                       array; values of the last substep
 *   carry[k]            device [rk_carry_rows(problem k)][n_sys[k]] controller state
 *                       carried from substep to substep and from call to call (see
 *                       rk_integrate_rkc_carry), or a NULL array: every substep a restart
 *   slot_map, n_total   interleaved form only (else NULL, 0)
 *   ws, ws_bytes        at least rk_batch_workspace_bytes(...), 256-byte aligned
 * Asynchronous on `stream`.  Calls on one batch must not overlap. */
int rk_batch_integrate_rkc(rk_batch b, const int64_t *n_sys, double *const *y,
                           const double *const *g, int32_t *const *status,
                           int32_t *const *stats, double *const *carry,
                           const int32_t *slot_map, int64_t n_total,
                           double t0, double dt, int32_t n_substeps, double rtol, double atol,
                           const rk_options *opt, const rk_batch_schedule *sched, void *ws,
                           size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif
#endif
