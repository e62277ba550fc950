/*
 * rk_oracle.h -- serial FP64 CPU oracle for batched RKCK / RKC integration.
 *
 * TEST INFRASTRUCTURE.  This is the plain, slow reference the GPU path is
 * checked against.  Only the test suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it; the product path never calls it.  It shares no
 * code with the GPU library.
 *
 * Method: Niemeyer & Sung, "GPU-Based Parallel Integration of Large Numbers of
 * Independent ODE Systems" (2014):
 *   Sec. 2       problem statement dy/dt = f(t, y, g), one system at a time
 *   Sec. 2.1     RKCK: Table 1 tableau, stage equations, error estimate,
 *                step-size rule (Eq. E:hnew) and the RKCK driver listing (Sec. 3.1)
 *   Sec. 2.2     RKC: stage recursion (Eqs. E:rkc0 - E:rkcs), coefficients,
 *                error estimate, RMS norm (Eq. E:rmsE), step-size rules
 *                (Eqs. dtnp1, rkc-f), initial step, stage count; the RKC driver
 *                listing (Sec. 3.2) and the nonlinear power method (Appendix)
 *   Sec. 4.2     mass-action species equations and Arrhenius rate coefficients
 *
 * Layout of batch arguments: struct-of-arrays, y[j*n + i] = unknown j of
 * system i (Sec. 3, column-major state storage).
 */
#ifndef RK_ORACLE_H
#define RK_ORACLE_H

#include <stdint.h>

#define ORC_MAXN 128      /* max unknowns per system */
#define ORC_MAXR 2048     /* max reactions */
#define ORC_MAXP 8        /* max per-system parameters */

enum { ORC_VDP = 1, ORC_LINEAR = 2, ORC_MASS_ACTION = 3, ORC_PLEIADES = 4,
       ORC_MASS_ACTION_THERMAL = 5 };

/* per-system status */
enum { ORC_OK = 0, ORC_NONFINITE = 1, ORC_HMIN = 2, ORC_MAXSTEPS = 3 };

/* Controller state carried from one call to the next instead of the restart
 * (Sec. 3 notes the alternative), rows of a per-system array followed by the
 * RKC eigenvector estimate (N rows); RKCK uses VALID and H.  VALID = 0 asks
 * for the restart; a call leaves VALID = 1 when its system ended OK. */
enum {
  ORC_CARRY_VALID = 0, ORC_CARRY_H, ORC_CARRY_H_PREV, ORC_CARRY_ERR_PREV, ORC_CARRY_SIGMA,
  ORC_CARRY_NSTEP, ORC_CARRY_HAVE_PREV, ORC_CARRY_ROWS
};

/* per-system statistics, SoA rows */
enum {
  ORC_ST_ACCEPT = 0,   /* accepted steps */
  ORC_ST_REJECT = 1,   /* rejected attempts */
  ORC_ST_RHS = 2,      /* right-hand-side evaluations */
  ORC_ST_SR_CALLS = 3, /* spectral-radius estimates (RKC) */
  ORC_ST_POW_ITERS = 4,/* power-method iterations (RKC) */
  ORC_ST_MAX_STAGES = 5,/* largest stage count used (RKC) */
  ORC_NSTATS = 6
};

typedef struct {
  int kind;            /* ORC_VDP | ORC_LINEAR | ORC_MASS_ACTION | ORC_PLEIADES */
  int n_eq;            /* N (Pleiades: 28) */
  int n_param;         /* entries of g per system: vdp 1 (mu), linear 0, mass action 2 (T, rho),
                          Pleiades 0, thermal mass action 1 (rho); n_eq = n_sp + 1 for the
                          thermal kind (row 0 is T) */
  const double *A;     /* ORC_LINEAR: f = A y, A row-major [N][N] */
  int n_rx;            /* ORC_MASS_ACTION: reactions */
  const int32_t *reac; /* [n_rx][2] species index per reactant slot, -1 = empty */
  const int32_t *prod; /* [n_rx][2] species index per product slot, -1 = empty */
  const double *lnA;   /* [n_rx] ln pre-exponential factor */
  const double *beta;  /* [n_rx] temperature exponent */
  const double *Ea;    /* [n_rx] activation temperature E/R, K */
  const double *Keq;   /* [n_rx] equilibrium constant k_f / k_r */
  const double *W;     /* [n_sp] molar masses */
  const double *thermo;/* ORC_MASS_ACTION_THERMAL: [3][n_sp] (u0, c, d): e_k(T) = u0 + (c + d T) T,
                          c_v,k(T) = c + 2 d T, per unit mass */
  int sr_method;       /* RKC spectral radius: 0 the nonlinear power method (Appendix),
                          1 the Gershgorin bound of the analytic Jacobian (ORC_VDP and
                          ORC_MASS_ACTION only) */
} orc_problem;

#ifdef __cplusplus
extern "C" {
#endif

/* Gershgorin bound max_k sum_i |J_ki| of J = df/dy at y for system g (ORC_VDP,
 * ORC_MASS_ACTION); J itself row-major into jac [N][N] when jac is not NULL.
 * Returns -1.0 for other problem kinds. */
double orc_gershgorin(const orc_problem *pb, const double *g, const double *y, double *jac);

/* ---- building blocks (exported so the tests can pin each one) ---- */
/* exp, log and pow correctly rounded (evaluated in binary128, rounded once) */
double orc_cr_exp(double x);
double orc_cr_log(double x);
double orc_cr_pow(double x, double y);
int  orc_n_theta(const orc_problem *pb);
void orc_rkck_tableau(double a[6], double b[36], double c[6], double cs[6], double e[6]);
int  orc_rhs(const orc_problem *pb, const double *g, double t, const double *y, double *f);
int  orc_rhs_vjp(const orc_problem *pb, const double *g, const double *y, const double *u,
                 double *jtu, double *dtheta);
int  orc_rkck_trial(const orc_problem *pb, const double *g, double t, const double *y,
                    const double *F, double h, double *ytemp, double *yerr);
double orc_rkck_error(int n, const double *y, const double *F, const double *yerr, double h,
                      double rtol, double atol, int *nan_flag);
double orc_rkck_control(double err, int nan_flag, double h, double hmin, double hmax,
                        int *accept);
int  orc_rkc_coeffs(int s, double *w0, double *w1, double *T, double *D, double *E,
                    double *b, double *a, double *mu, double *nu, double *mut, double *gt,
                    double *c);
int  orc_rkc_step(const orc_problem *pb, const double *g, double t, const double *y,
                  const double *F, double h, int s, double *yout);
int  orc_rkc_stages(const orc_problem *pb, const double *g, double t, const double *y,
                    const double *F, double h, int s, double *W);
double orc_spec_rad(const orc_problem *pb, const double *g, double t, const double *y,
                    const double *F, double hmax, double *v, int itmax, int *iters);
int  orc_rkc_mmax(double rtol);
int  orc_rkc_stage_count(double h, double sigma, int mmax, double *h_out);
double orc_rkc_accept_factor(double err, double err_prev, double h, double h_prev,
                             int have_prev);

/* ---- whole integrations, one system ---- */
int orc_rkck_solve(const orc_problem *pb, const double *g, const double *y0, double *y1,
                   double t0, double t1, double rtol, double atol, int64_t max_steps,
                   int32_t *stats);
/* As orc_rkck_solve; rec_h (capacity rec_cap) receives the accepted steps'
 * sizes, *n_rec their number (may exceed rec_cap: not stored). */
int orc_rkck_solve_rec(const orc_problem *pb, const double *g, const double *y0, double *y1,
                       double t0, double t1, double rtol, double atol, int64_t max_steps,
                       int32_t *stats, double *rec_h, int64_t rec_cap, int64_t *n_rec);
/* rec_h / rec_s (capacity rec_cap, may be NULL) receive the accepted steps'
 * size and stage count; *n_rec their number (may exceed rec_cap: not stored). */
int orc_rkc_solve(const orc_problem *pb, const double *g, const double *y0, double *y1,
                  double t0, double t1, double rtol, double atol, int64_t max_steps,
                  int32_t *stats, double *rec_h, int32_t *rec_s, int64_t rec_cap,
                  int64_t *n_rec);
/* One attempted RKC step, as the driver made it (orc_rkc_solve_trace). */
typedef struct {
  double t;        /* time at the start of the attempt */
  double h_want;   /* step the controller proposed (before the end-point stretch) */
  double h;        /* step taken (after the stretch, the initial-step rule, the stage cap) */
  double sigma;    /* spectral radius used for the stage count */
  double err;      /* weighted RMS error of the attempt */
  int64_t nstep;   /* accepted steps before the attempt */
  int64_t n_sr;    /* spectral-radius estimates made so far, this attempt's included */
  int32_t m;       /* stages */
  int32_t accepted;
} orc_rkc_attempt;
/* As orc_rkc_solve; trace (capacity trace_cap) receives one record per
 * attempt, *n_trace the number of attempts (may exceed trace_cap). */
int orc_rkc_solve_trace(const orc_problem *pb, const double *g, const double *y0, double *y1,
                        double t0, double t1, double rtol, double atol, int64_t max_steps,
                        int32_t *stats, orc_rkc_attempt *trace, int64_t trace_cap,
                        int64_t *n_trace);
/* Replays accepted RKC steps (h_k, s_k) from y0 with no controller. */
int orc_rkc_replay(const orc_problem *pb, const double *g, const double *y0, double t0,
                   int64_t n_steps, const double *h, const int32_t *s, double *y1);
/* Discrete adjoint of the replayed accepted-step map for L = w . y(t1):
 * dy0 = dL/dy0 [N], dtheta = dL/dtheta [orc_n_theta]. */
int orc_rkc_replay_adjoint(const orc_problem *pb, const double *g, const double *y0,
                           double t0, int64_t n_steps, const double *h, const int32_t *s,
                           const double *w, double *dy0, double *dtheta);
/* Replays accepted RKCK steps h_k from y0 with no controller. */
int orc_rkck_replay(const orc_problem *pb, const double *g, const double *y0, double t0,
                    int64_t n_steps, const double *h, double *y1);
/* Discrete adjoint of the replayed RKCK step map for L = w . y(t1). */
int orc_rkck_replay_adjoint(const orc_problem *pb, const double *g, const double *y0,
                            double t0, int64_t n_steps, const double *h, const double *w,
                            double *dy0, double *dtheta);

/* Complex-step directional derivatives of L = w . y(t1) along (dy0, dtheta)
 * for the replayed RKC / RKCK step maps (ORC_VDP, ORC_LINEAR, ORC_MASS_ACTION):
 * Im L(y0 + i e dy0, theta + i e dtheta) / e with e = 1e-20, every operation of
 * the replay carried out in complex arithmetic; free of the cancellation of
 * finite differences.  dtheta has orc_n_theta entries (may be NULL: zero). */
int orc_rkc_replay_jvp_cs(const orc_problem *pb, const double *g, const double *y0, double t0,
                          int64_t n_steps, const double *h, const int32_t *s, const double *w,
                          const double *dy0, const double *dtheta, double *jvp);
int orc_rkck_replay_jvp_cs(const orc_problem *pb, const double *g, const double *y0, double t0,
                           int64_t n_steps, const double *h, const double *w, const double *dy0,
                           const double *dtheta, double *jvp);

/* ---- batches (SoA), OpenMP across systems; n_threads <= 0: runtime default ---- */
int orc_rkck_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                   double *y1, double t0, double t1, double rtol, double atol,
                   int64_t max_steps, int32_t *status, int32_t *stats, int n_threads);
int orc_rkc_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                  double *y1, double t0, double t1, double rtol, double atol,
                  int64_t max_steps, int32_t *status, int32_t *stats, int n_threads);
/* forward RKC + adjoint per system; dy0 [N][n], dtheta [n_theta][n] SoA */
int orc_rkc_adjoint_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                          double t0, double t1, double rtol, double atol, int64_t max_steps,
                          const double *w, double *y1, double *dy0, double *dtheta,
                          int32_t *status, int n_threads);
/* forward RKCK + adjoint per system, as orc_rkc_adjoint_batch */
int orc_rkck_adjoint_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                           double t0, double t1, double rtol, double atol, int64_t max_steps,
                           const double *w, double *y1, double *dy0, double *dtheta,
                           int32_t *status, int n_threads);
int orc_rkck_batch_carry(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                         double *y1, double t0, double t1, double rtol, double atol,
                         int64_t max_steps, int32_t *status, int32_t *stats, double *carry,
                         int n_threads);
int orc_rkc_batch_carry(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                        double *y1, double t0, double t1, double rtol, double atol,
                        int64_t max_steps, int32_t *status, int32_t *stats, double *carry,
                        int n_threads);
int orc_max_threads(void);

#ifdef __cplusplus
}
#endif
#endif
