/*
 * rk_oracle.c -- serial FP64 CPU oracle for batched RKCK / RKC integration.
 *
 * TEST INFRASTRUCTURE (see rk_oracle.h).  Plain loops, one system at a time,
 * in the order the paper states each step; built with -O2 -ffp-contract=off so
 * every operation rounds once, as written.  Shares no code with the GPU path.
 *
 * Readings taken where the paper is silent, garbled or inconsistent are marked
 * "Reading:" at the place they apply.
 */
#include "rk_oracle.h"

#include <complex.h>
#include <math.h>
#include <quadmath.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------- transcendentals
 * Reading: the paper does not say how accurately exp, log and pow are
 * evaluated.  Step-size and stage-count decisions hinge on their last bit, so
 * the oracle evaluates each one correctly rounded: the exact value rounded to
 * the nearest double, obtained by evaluating in IEEE binary128 (libquadmath)
 * and rounding once to double.  Special values follow C99 Annex F. */
double orc_cr_exp(double x) {
  if (isnan(x)) return x;
  return (double)expq((__float128)x);
}

double orc_cr_log(double x) {
  if (isnan(x)) return x;
  if (x < 0.0) return NAN;
  if (x == 0.0) return -INFINITY;
  if (isinf(x)) return x;
  return (double)logq((__float128)x);
}

double orc_cr_pow(double x, double y) {
  if (y == 0.0 || x == 1.0) return 1.0;
  if (isnan(x) || isnan(y)) return x + y;
  return (double)powq((__float128)x, (__float128)y);
}

/* Constants of the RKCK driver (Sec. 3.1 constant list). */
#define UROUND 2.22e-16
#define SAFETY 0.9
#define PGROW (-0.2)
#define PSHRNK (-0.25)
#define ERRCON 1.89e-4
#define TINY 1.0e-30
/* Reading: the factor P1 is used but never defined in the listings; the text
 * limits step decreases to a factor of ten (Sec. 2.1) and bounds the RKC factor
 * below by 0.1 (Eq. dtnp1), so P1 = 0.1. */
#define P1 0.1

/* ------------------------------------------------------------------ systems */

/* One system's view of the problem: its parameters g and, for mass action,
 * its rate coefficients, computed once because T is constant (isothermal). */
typedef struct {
  const orc_problem *pb;
  double g[ORC_MAXP];
  double kf[ORC_MAXR];
  double kr[ORC_MAXR];
  double invW[ORC_MAXN];
  double rho, irho;
} orc_sys;

static int check_problem(const orc_problem *pb) {
  if (!pb || pb->n_eq <= 0 || pb->n_eq > ORC_MAXN || pb->n_param < 0 || pb->n_param > ORC_MAXP)
    return -1;
  if (pb->kind == ORC_VDP && (pb->n_eq != 2 || pb->n_param < 1)) return -1;
  if (pb->kind == ORC_LINEAR && !pb->A) return -1;
  if (pb->kind == ORC_MASS_ACTION &&
      (pb->n_rx <= 0 || pb->n_rx > ORC_MAXR || pb->n_param < 2 || !pb->reac || !pb->prod ||
       !pb->lnA || !pb->beta || !pb->Ea || !pb->Keq || !pb->W))
    return -1;
  if (pb->kind == ORC_PLEIADES && pb->n_eq != 28) return -1;
  if (pb->kind == ORC_MASS_ACTION_THERMAL &&
      (pb->n_eq < 2 || pb->n_rx <= 0 || pb->n_rx > ORC_MAXR || pb->n_param < 1 || !pb->reac ||
       !pb->prod || !pb->lnA || !pb->beta || !pb->Ea || !pb->Keq || !pb->W || !pb->thermo))
    return -1;
  if (pb->kind != ORC_VDP && pb->kind != ORC_LINEAR && pb->kind != ORC_MASS_ACTION &&
      pb->kind != ORC_PLEIADES && pb->kind != ORC_MASS_ACTION_THERMAL)
    return -1;
  if (pb->sr_method != 0 &&
      (pb->sr_method != 1 || (pb->kind != ORC_VDP && pb->kind != ORC_MASS_ACTION) || pb->n_eq > 16))
    return -1;
  return 0;
}

/* Problems with vector-Jacobian products (every kind but Pleiades). */
static int check_vjp_problem(const orc_problem *pb) {
  return (check_problem(pb) || pb->kind == ORC_PLEIADES || pb->kind == ORC_MASS_ACTION_THERMAL)
             ? -1
             : 0;
}

/* Arrhenius rate coefficient k = A T^beta exp(-E/T) (Sec. 4.2), evaluated in
 * log form so that ln A enters additively; reverse k_r = k_f / K.  The
 * divisions by the constants K_j, W_k and rho are written as multiplications
 * by their reciprocals, each formed once (per network or per system). */
static void sys_init(orc_sys *S, const orc_problem *pb, const double *g) {
  S->pb = pb;
  for (int i = 0; i < pb->n_param; ++i) S->g[i] = g[i];
  if (pb->kind == ORC_MASS_ACTION_THERMAL) {
    S->rho = g[0];
    S->irho = 1.0 / S->rho;
    for (int k = 0; k < pb->n_eq - 1; ++k) S->invW[k] = 1.0 / pb->W[k];
  }
  if (pb->kind == ORC_MASS_ACTION) {
    double T = g[0];
    double lnT = orc_cr_log(T);
    S->rho = g[1];
    S->irho = 1.0 / S->rho;
    for (int k = 0; k < pb->n_eq; ++k) S->invW[k] = 1.0 / pb->W[k];
    for (int j = 0; j < pb->n_rx; ++j) {
      S->kf[j] = orc_cr_exp(pb->lnA[j] + pb->beta[j] * lnT - pb->Ea[j] / T);
      S->kr[j] = S->kf[j] * (1.0 / pb->Keq[j]);
    }
  }
}

/* Right-hand side f(t, y, g) of Eq. (1).  Every problem here is autonomous. */
static void rhs(const orc_sys *S, double t, const double *y, double *f) {
  const orc_problem *pb = S->pb;
  const int N = pb->n_eq;
  (void)t;
  if (pb->kind == ORC_VDP) {
    double mu = S->g[0];
    f[0] = y[1];
    f[1] = mu * (1.0 - y[0] * y[0]) * y[1] - y[0];
  } else if (pb->kind == ORC_LINEAR) {
    for (int i = 0; i < N; ++i) {
      double s = 0.0;
      for (int j = 0; j < N; ++j) s += pb->A[i * N + j] * y[j];
      f[i] = s;
    }
  } else if (pb->kind == ORC_MASS_ACTION_THERMAL) {
    /* Non-isothermal species equations at constant volume (Sec. 4.2): state
     * (T, Y_1..Y_N);
     *   dY_k/dt = W_k omega_k / rho,
     *   dT/dt = -(1 / (rho c_v)) sum_k e_k omega_k W_k,  c_v = sum_k Y_k c_v,k(T),
     * with the rate coefficients evaluated at the current T on every call,
     * k_f,j = exp(ln A_j + beta_j ln T - Ea_j / T), k_r,j = k_f,j / K_j, and
     * the synthetic per-mass internal energies e_k(T) = u0_k + (c_k + d_k T) T,
     * c_v,k(T) = c_k + 2 d_k T.  Readings as the isothermal rate law (left to
     * right, reciprocals of constants), plus: Ea_j / T as Ea_j times 1 / T
     * formed once per call; the energy sum accumulated (e_k omega_k) W_k from
     * zero in species order and scaled as -((sum / rho) / c_v) with 1 / rho. */
    const int NS = N - 1;
    const double T = y[0];
    const double lnT = orc_cr_log(T);
    const double invT = 1.0 / T;
    const double *u0 = pb->thermo, *cc = pb->thermo + NS, *dd = pb->thermo + 2 * NS;
    double kf[ORC_MAXR], kr[ORC_MAXR], C[ORC_MAXN], omega[ORC_MAXN];
    for (int j = 0; j < pb->n_rx; ++j) {
      kf[j] = orc_cr_exp(pb->lnA[j] + pb->beta[j] * lnT - pb->Ea[j] * invT);
      kr[j] = kf[j] * (1.0 / pb->Keq[j]);
    }
    double M = 0.0;
    for (int k = 0; k < NS; ++k) C[k] = (S->rho * y[1 + k]) * S->invW[k];
    for (int k = 0; k < NS; ++k) M += C[k];
    for (int k = 0; k < NS; ++k) omega[k] = 0.0;
    for (int j = 0; j < pb->n_rx; ++j) {
      int r0 = pb->reac[2 * j], r1 = pb->reac[2 * j + 1];
      int p0 = pb->prod[2 * j], p1 = pb->prod[2 * j + 1];
      double fwd = kf[j] * C[r0] * (r1 >= 0 ? C[r1] : M);
      double rev = kr[j] * C[p0] * (p1 >= 0 ? C[p1] : M);
      double q = fwd - rev;
      omega[r0] -= q;
      if (r1 >= 0) omega[r1] -= q;
      omega[p0] += q;
      if (p1 >= 0) omega[p1] += q;
    }
    for (int k = 0; k < NS; ++k) f[1 + k] = (pb->W[k] * omega[k]) * S->irho;
    double sum = 0.0, cv = 0.0;
    for (int k = 0; k < NS; ++k) {
      const double e = u0[k] + (cc[k] + dd[k] * T) * T;
      sum += (e * omega[k]) * pb->W[k];
      cv += y[1 + k] * (cc[k] + 2.0 * dd[k] * T);
    }
    f[0] = -((sum * S->irho) / cv);
  } else if (pb->kind == ORC_PLEIADES) {
    /* Pleiades problem (Sec. 4.1): seven bodies of mass m_i = i (1-based) in the
     * plane, state (x_1..x_7, y_1..y_7, x_1'..x_7', y_1'..y_7'); z'' = f(z) as
     * the 28 first-order equations (z, w)' = (w, f(z)):
     *   x_i'' = sum_{j != i} m_j (x_j - x_i) / r_ij,  y_i'' likewise,
     *   r_ij = ((x_i - x_j)^2 + (y_i - y_j)^2)^(3/2).
     * Readings: the y difference is squared (the printed formula drops the
     * square); the 3/2 power is d2 * sqrt(d2) with d2 the sum of squares; the
     * division by r_ij is a multiplication by 1 / r_ij; each sum runs over j in
     * increasing order from zero. */
    const double *x = y, *yy = y + 7;
    for (int i = 0; i < 14; ++i) f[i] = y[14 + i];
    for (int i = 0; i < 7; ++i) {
      double ax = 0.0, ay = 0.0;
      for (int j = 0; j < 7; ++j) {
        if (j == i) continue;
        const double mj = (double)(j + 1);
        const double d2 = (x[i] - x[j]) * (x[i] - x[j]) + (yy[i] - yy[j]) * (yy[i] - yy[j]);
        const double rinv = 1.0 / (d2 * sqrt(d2));
        ax += (mj * (x[j] - x[i])) * rinv;
        ay += (mj * (yy[j] - yy[i])) * rinv;
      }
      f[14 + i] = ax;
      f[21 + i] = ay;
    }
  } else {
    /* Species equations of Sec. 4.2 at constant T: dY_k/dt = W_k omega_k / rho,
     * omega_k = sum_j nu_kj q_j, C_k = rho Y_k / W_k.  Convention for this
     * synthetic network: reversible reactions, q_j = k_f prod_R C - k_r prod_P C,
     * a one-species side multiplied by the total concentration [M].  Both
     * conversions are evaluated left to right as written, (rho Y_k) / W_k and
     * (W_k omega_k) / rho, each division by a constant of the system being a
     * multiplication by its reciprocal. */
    double C[ORC_MAXN], omega[ORC_MAXN];
    double M = 0.0;
    for (int k = 0; k < N; ++k) C[k] = (S->rho * y[k]) * S->invW[k];
    for (int k = 0; k < N; ++k) M += C[k];
    for (int k = 0; k < N; ++k) omega[k] = 0.0;
    for (int j = 0; j < pb->n_rx; ++j) {
      int r0 = pb->reac[2 * j], r1 = pb->reac[2 * j + 1];
      int p0 = pb->prod[2 * j], p1 = pb->prod[2 * j + 1];
      double fwd = S->kf[j] * C[r0] * (r1 >= 0 ? C[r1] : M);
      double rev = S->kr[j] * C[p0] * (p1 >= 0 ? C[p1] : M);
      double q = fwd - rev;
      omega[r0] -= q;
      if (r1 >= 0) omega[r1] -= q;
      omega[p0] += q;
      if (p1 >= 0) omega[p1] += q;
    }
    for (int k = 0; k < N; ++k) f[k] = (pb->W[k] * omega[k]) * S->irho;
  }
}

/* Analytic Jacobian J = df/dy of Eq. (1) at y and its Gershgorin bound.  The
 * Appendix names the circle theorem as an alternative to the power method: every
 * eigenvalue lies in a disc |z - J_kk| <= sum_{i != k} |J_ki|, so the spectral
 * radius is at most max_k sum_i |J_ki|.  Readings: rows k in order, each row sum
 * over i in order from zero, the maximum by fmax from zero; the bound is used as
 * sigma as it is (it needs no safety factor).
 *   van der Pol: J = [[0, 1], [-2 mu y_0 y_1 - 1, mu (1 - y_0^2)]], left to right.
 *   mass action (isothermal): with C_i = rho Y_i / W_i, [M] = sum_i C_i and
 *   q_j = (k_f C_r0) X_r1 - (k_r C_p0) X_p1 (X = C, or [M] for an empty slot),
 *   J_ki = (W_k D_ki) / W_i (the rho factors cancel; the division as the
 *   reciprocal), D_ki = sum_j nu_kj g_ji over the reactions in order with
 *   nu_kj = (products - reactants) count of k nonzero, and
 *   g_ji = dq_j/dC_i through C_i and [M]: k_f t_f - k_r t_r with
 *   t_f = [r0 = i] X_r1 + [r1 = i or empty] C_r0 (terms absent where zero),
 *   t_r likewise. */
static void jacobian(const orc_sys *S, const double *y, double *J) {
  const orc_problem *pb = S->pb;
  const int N = pb->n_eq;
  if (pb->kind == ORC_VDP) {
    const double mu = S->g[0];
    J[0] = 0.0;
    J[1] = 1.0;
    J[2] = -2.0 * mu * y[0] * y[1] - 1.0;
    J[3] = mu * (1.0 - y[0] * y[0]);
    return;
  }
  double C[ORC_MAXN];
  double M = 0.0;
  for (int k = 0; k < N; ++k) C[k] = (S->rho * y[k]) * S->invW[k];
  for (int k = 0; k < N; ++k) M += C[k];
  for (int k = 0; k < N; ++k)
    for (int i = 0; i < N; ++i) {
      double D = 0.0;
      for (int j = 0; j < pb->n_rx; ++j) {
        const int r0 = pb->reac[2 * j], r1 = pb->reac[2 * j + 1];
        const int p0 = pb->prod[2 * j], p1 = pb->prod[2 * j + 1];
        const int nu = (p0 == k) + (p1 == k) - (r0 == k) - (r1 == k);
        if (nu == 0) continue;
        const double xr1 = r1 >= 0 ? C[r1] : M, xp1 = p1 >= 0 ? C[p1] : M;
        const double tf = (r0 == i ? xr1 : 0.0) + ((r1 < 0 || r1 == i) ? C[r0] : 0.0);
        const double tr = (p0 == i ? xp1 : 0.0) + ((p1 < 0 || p1 == i) ? C[p0] : 0.0);
        D += (double)nu * (S->kf[j] * tf - S->kr[j] * tr);
      }
      J[k * N + i] = (pb->W[k] * D) * S->invW[i];
    }
}

static double gershgorin(const orc_sys *S, const double *y, double *Jout) {
  const int N = S->pb->n_eq;
  double Jl[ORC_MAXN * 16];
  double *J = Jout ? Jout : Jl;
  jacobian(S, y, J);
  double sigma = 0.0;
  for (int k = 0; k < N; ++k) {
    double r = 0.0;
    for (int i = 0; i < N; ++i) r += fabs(J[k * N + i]);
    sigma = fmax(sigma, r);
  }
  return sigma;
}

double orc_gershgorin(const orc_problem *pb, const double *g, const double *y, double *jac) {
  if (check_problem(pb) || (pb->kind != ORC_VDP && pb->kind != ORC_MASS_ACTION) || pb->n_eq > 16)
    return -1.0;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -1.0;
  sys_init(S, pb, g);
  const double s = gershgorin(S, y, jac);
  free(S);
  return s;
}

int orc_n_theta(const orc_problem *pb) {
  if (!pb) return 0;
  if (pb->kind == ORC_VDP) return 1;                  /* mu */
  if (pb->kind == ORC_MASS_ACTION) return pb->n_rx;   /* ln A_j */
  return 0;
}

/* Vector-Jacobian products of f: jtu = J(y)^T u and dtheta = (df/dtheta)^T u,
 * theta = mu (van der Pol) or ln A (mass action). */
static void rhs_vjp(const orc_sys *S, const double *y, const double *u, double *jtu,
                    double *dtheta) {
  const orc_problem *pb = S->pb;
  const int N = pb->n_eq;
  if (pb->kind == ORC_VDP) {
    double mu = S->g[0];
    jtu[0] = u[1] * (-2.0 * mu * y[0] * y[1] - 1.0);
    jtu[1] = u[0] + u[1] * mu * (1.0 - y[0] * y[0]);
    dtheta[0] = u[1] * (1.0 - y[0] * y[0]) * y[1];
  } else if (pb->kind == ORC_LINEAR) {
    for (int j = 0; j < N; ++j) {
      double s = 0.0;
      for (int i = 0; i < N; ++i) s += pb->A[i * N + j] * u[i];
      jtu[j] = s;
    }
  } else {
    double C[ORC_MAXN], uw[ORC_MAXN], Cbar[ORC_MAXN];
    double M = 0.0, Mbar = 0.0;
    for (int k = 0; k < N; ++k) C[k] = (S->rho * y[k]) * S->invW[k];
    for (int k = 0; k < N; ++k) M += C[k];
    /* u^T f = sum_k (W_k/rho) u_k omega_k */
    for (int k = 0; k < N; ++k) uw[k] = (pb->W[k] * S->irho) * u[k];
    for (int k = 0; k < N; ++k) Cbar[k] = 0.0;
    for (int j = 0; j < pb->n_rx; ++j) {
      int r0 = pb->reac[2 * j], r1 = pb->reac[2 * j + 1];
      int p0 = pb->prod[2 * j], p1 = pb->prod[2 * j + 1];
      /* r = d(u^T f)/d q_j = sum_k nu_kj uw_k */
      double r = -uw[r0] + (r1 >= 0 ? -uw[r1] : 0.0) + uw[p0] + (p1 >= 0 ? uw[p1] : 0.0);
      double fwd = S->kf[j] * C[r0] * (r1 >= 0 ? C[r1] : M);
      double rev = S->kr[j] * C[p0] * (p1 >= 0 ? C[p1] : M);
      /* both k_f and k_r are proportional to A_j: dq/dlnA = q */
      dtheta[j] = r * (fwd - rev);
      /* forward product */
      double a = r * S->kf[j];
      if (r1 >= 0) {
        Cbar[r0] += a * C[r1];
        Cbar[r1] += a * C[r0];
      } else {
        Cbar[r0] += a * M;
        Mbar += a * C[r0];
      }
      double b = -r * S->kr[j];
      if (p1 >= 0) {
        Cbar[p0] += b * C[p1];
        Cbar[p1] += b * C[p0];
      } else {
        Cbar[p0] += b * M;
        Mbar += b * C[p0];
      }
    }
    /* d M / d C_k = 1, d C_k / d y_k = rho / W_k */
    for (int k = 0; k < N; ++k) jtu[k] = (S->rho * S->invW[k]) * (Cbar[k] + Mbar);
  }
}

int orc_rhs(const orc_problem *pb, const double *g, double t, const double *y, double *f) {
  if (check_problem(pb)) return -1;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -2;
  sys_init(S, pb, g);
  rhs(S, t, y, f);
  free(S);
  return 0;
}

int orc_rhs_vjp(const orc_problem *pb, const double *g, const double *y, const double *u,
                double *jtu, double *dtheta) {
  if (check_vjp_problem(pb)) return -1;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -2;
  sys_init(S, pb, g);
  double dummy[1];
  rhs_vjp(S, y, u, jtu, orc_n_theta(pb) ? dtheta : dummy);
  free(S);
  return 0;
}

static int all_finite(int n, const double *y) {
  for (int i = 0; i < n; ++i)
    if (!isfinite(y[i])) return 0;
  return 1;
}

/* ===================================================================== RKCK */

/* Table 1: Cash-Karp coefficients, stage nodes a_i, couplings b_ij, fifth-order
 * weights c_i and embedded fourth-order weights c*_i; every entry is the
 * nearest double of the printed fraction. */
static const double RKCK_A[6] = {0.0, 1.0 / 5.0, 3.0 / 10.0, 3.0 / 5.0, 1.0, 7.0 / 8.0};
static const double RKCK_B[6][5] = {
    {0.0, 0.0, 0.0, 0.0, 0.0},
    {1.0 / 5.0, 0.0, 0.0, 0.0, 0.0},
    {3.0 / 40.0, 9.0 / 40.0, 0.0, 0.0, 0.0},
    {3.0 / 10.0, -9.0 / 10.0, 6.0 / 5.0, 0.0, 0.0},
    {-11.0 / 54.0, 5.0 / 2.0, -70.0 / 27.0, 35.0 / 27.0, 0.0},
    {1631.0 / 55296.0, 175.0 / 512.0, 575.0 / 13824.0, 44275.0 / 110592.0, 253.0 / 4096.0}};
static const double RKCK_C[6] = {37.0 / 378.0, 0.0, 250.0 / 621.0, 125.0 / 594.0, 0.0,
                                 512.0 / 1771.0};
static const double RKCK_CS[6] = {2825.0 / 27648.0, 0.0, 18575.0 / 48384.0,
                                  13525.0 / 55296.0, 277.0 / 14336.0, 1.0 / 4.0};
/* Error weights c_i - c*_i of the local error estimate (Sec. 2.1), each the
 * nearest double of the exact rational difference. */
static const double RKCK_E[6] = {-277.0 / 64512.0, 0.0, 6925.0 / 370944.0,
                                 -6925.0 / 202752.0, -277.0 / 14336.0, 277.0 / 7084.0};

void orc_rkck_tableau(double a[6], double b[36], double c[6], double cs[6], double e[6]) {
  for (int i = 0; i < 6; ++i) {
    a[i] = RKCK_A[i];
    c[i] = RKCK_C[i];
    cs[i] = RKCK_CS[i];
    e[i] = RKCK_E[i];
    for (int j = 0; j < 6; ++j) b[i * 6 + j] = (j < 5) ? RKCK_B[i][j] : 0.0;
  }
}

/* One RKCK trial step (Sec. 2.1 stage equations): k_1 = h F with F = f(t, y)
 * supplied; k_i = h f(t + a_i h, y + sum_{j<i} b_ij k_j); the fifth-order
 * solution y + sum c_i k_i and the error estimate sum (c_i - c*_i) k_i. */
static void rkck_trial_z(const orc_sys *S, double t, const double *y, const double *F, double h,
                         double *ytemp, double *yerr, double *zst) {
  const int N = S->pb->n_eq;
  double k[6][ORC_MAXN], z[ORC_MAXN], f[ORC_MAXN];
  for (int i = 0; i < N; ++i) k[0][i] = h * F[i];
  if (zst)
    for (int i = 0; i < N; ++i) zst[i] = y[i];
  for (int s = 1; s < 6; ++s) {
    for (int i = 0; i < N; ++i) {
      double acc = y[i];
      for (int j = 0; j < s; ++j) acc = acc + RKCK_B[s][j] * k[j][i];
      z[i] = acc;
    }
    if (zst)
      for (int i = 0; i < N; ++i) zst[(size_t)s * N + i] = z[i];
    rhs(S, t + RKCK_A[s] * h, z, f);
    for (int i = 0; i < N; ++i) k[s][i] = h * f[i];
  }
  /* weights that are zero in Table 1 (c_2, c_5, and c_2 - c*_2) contribute
   * nothing and are skipped */
  for (int i = 0; i < N; ++i) {
    double acc = y[i];
    for (int s = 0; s < 6; ++s)
      if (RKCK_C[s] != 0.0) acc = acc + RKCK_C[s] * k[s][i];
    ytemp[i] = acc;
    double e = 0.0;
    for (int s = 0; s < 6; ++s)
      if (RKCK_E[s] != 0.0) e = e + RKCK_E[s] * k[s][i];
    yerr[i] = e;
  }
}

static void rkck_trial(const orc_sys *S, double t, const double *y, const double *F, double h,
                       double *ytemp, double *yerr) {
  rkck_trial_z(S, t, y, F, h, ytemp, yerr, NULL);
}

int orc_rkck_trial(const orc_problem *pb, const double *g, double t, const double *y,
                   const double *F, double h, double *ytemp, double *yerr) {
  if (check_problem(pb)) return -1;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -2;
  sys_init(S, pb, g);
  rkck_trial(S, t, y, F, h, ytemp, yerr);
  free(S);
  return 0;
}

/* Scaled error of an RKCK trial (Sec. 2.1 desired accuracy; listing of the
 * RKCK driver): err = max_i |yerr_i / (|y_i| + |h F_i| + delta)| / eps.
 * Reading: eps is the relative tolerance rtol and delta = atol / rtol, so the
 * scale is rtol (|y| + |h F|) + atol; with atol = 0, delta is TINY.
 * fmax ignores NaN, hence the separate NaN flag. */
double orc_rkck_error(int n, const double *y, const double *F, const double *yerr, double h,
                      double rtol, double atol, int *nan_flag) {
  double delta = (atol > 0.0) ? atol / rtol : TINY;
  double err = 0.0;
  int nan = 0;
  for (int i = 0; i < n; ++i) {
    if (isnan(yerr[i])) nan = 1;
    err = fmax(err, fabs(yerr[i] / (fabs(y[i]) + fabs(h * F[i]) + delta)));
  }
  if (nan_flag) *nan_flag = nan;
  return err / rtol;
}

/* RKCK step-size rule (Eq. E:hnew with the driver listing's constants).
 * Reading: the listing's form is used, err^(-1/5) and err^(-1/4) with err the
 * max over components of |Delta/Delta0|; the equation's max of the inverse
 * ratio would select the least-constrained component.  Returns the new step
 * and sets *accept. */
double orc_rkck_control(double err, int nan_flag, double h, double hmin, double hmax,
                        int *accept) {
  if ((err > 1.0) || isnan(err) || nan_flag) {
    *accept = 0;
    if (isnan(err) || nan_flag) return h * P1;
    return fmax(SAFETY * h * orc_cr_pow(err, PSHRNK), P1 * h);
  }
  *accept = 1;
  double hn;
  if (err > ERRCON)
    hn = SAFETY * h * orc_cr_pow(err, PGROW);
  else
    hn = h * 5.0;
  return fmax(hmin, fmin(hmax, hn));
}

/* Record of the accepted steps of one integration: (h, s) per step; grows by
 * realloc when `grow` is set, else keeps the first cap steps and counts the rest. */
typedef struct {
  double *h;
  int32_t *s;
  int64_t n, cap;
  int grow; /* 1: realloc as needed */
} step_rec;

static void rec_push(step_rec *r, double h, int s) {
  if (!r) return;
  if (r->n >= r->cap && r->grow) {
    int64_t nc = r->cap ? 2 * r->cap : 256;
    double *nh = (double *)realloc(r->h, sizeof(double) * nc);
    if (nh) r->h = nh;
    int32_t *ns = (int32_t *)realloc(r->s, sizeof(int32_t) * nc);
    if (ns) r->s = ns;
    if (nh && ns) r->cap = nc;
  }
  if (r->n < r->cap && r->h && r->s) {
    r->h[r->n] = h;
    r->s[r->n] = s;
  }
  r->n++;
}

/* RKCK driver (Sec. 3.1): hMax = |t1 - t0|, hMin = 1e-20, first trial step
 * half the interval; loop until t reaches t1, clipping the step to the time
 * left.  Reading: f(t, y) is kept after a rejection (same arguments, same
 * value) instead of being evaluated again; guards stop a system whose step
 * falls below hMin after a rejection, whose accepted state is not finite, or
 * that exhausts max_steps attempts (the listing has no exit for these). */
static int rkck_solve_impl(const orc_problem *pb, const double *g, const double *y0, double *y1,
                           double t0, double t1, double rtol, double atol, int64_t max_steps,
                           int32_t *stats, step_rec *rec, double *carry) {
  if (check_problem(pb) || !(t1 >= t0) || !(rtol > 0.0) || !(atol >= 0.0)) return -1;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -2;
  sys_init(S, pb, g);
  const int N = pb->n_eq;
  double y[ORC_MAXN], F[ORC_MAXN], ytemp[ORC_MAXN], yerr[ORC_MAXN];
  for (int i = 0; i < N; ++i) y[i] = y0[i];
  double t = t0;
  const double hmax = fabs(t1 - t0);
  const double hmin = 1.0e-20;
  double h = 0.5 * fabs(t1 - t0);
  /* a carried state brings the step the previous call would have taken next */
  if (carry && carry[ORC_CARRY_VALID] != 0.0) h = carry[ORC_CARRY_H];
  double h_want = h;
  int cut = 0;
  int fvalid = 0, status = ORC_OK;
  int64_t attempts = 0, n_acc = 0, n_rej = 0, n_rhs = 0;
  while (t < t1) {
    if (attempts >= max_steps) {
      status = ORC_MAXSTEPS;
      break;
    }
    h_want = h;
    h = fmin(t1 - t, h);
    if (!fvalid) {
      rhs(S, t, y, F);
      n_rhs++;
      fvalid = 1;
    }
    rkck_trial(S, t, y, F, h, ytemp, yerr);
    n_rhs += 5;
    int nan_flag = 0, accept = 0;
    double err = orc_rkck_error(N, y, F, yerr, h, rtol, atol, &nan_flag);
    double hnew = orc_rkck_control(err, nan_flag, h, hmin, hmax, &accept);
    attempts++;
    if (!accept) {
      n_rej++;
      h = hnew;
      if (!(h >= hmin)) {
        status = ORC_HMIN;
        break;
      }
    } else {
      cut = h < h_want;
      rec_push(rec, h, 6);
      t += h;
      h = hnew;
      for (int i = 0; i < N; ++i) y[i] = ytemp[i];
      n_acc++;
      fvalid = 0;
      if (!all_finite(N, y)) {
        status = ORC_NONFINITE;
        break;
      }
    }
  }
  if (carry) {
    carry[ORC_CARRY_VALID] = status == ORC_OK ? 1.0 : 0.0;
    carry[ORC_CARRY_H] = cut ? h_want : h;
  }
  for (int i = 0; i < N; ++i) y1[i] = y[i];
  if (stats) {
    stats[ORC_ST_ACCEPT] = (int32_t)n_acc;
    stats[ORC_ST_REJECT] = (int32_t)n_rej;
    stats[ORC_ST_RHS] = (int32_t)n_rhs;
    stats[ORC_ST_SR_CALLS] = 0;
    stats[ORC_ST_POW_ITERS] = 0;
    stats[ORC_ST_MAX_STAGES] = 6;
  }
  free(S);
  return status;
}

int orc_rkck_solve(const orc_problem *pb, const double *g, const double *y0, double *y1,
                   double t0, double t1, double rtol, double atol, int64_t max_steps,
                   int32_t *stats) {
  return rkck_solve_impl(pb, g, y0, y1, t0, t1, rtol, atol, max_steps, stats, NULL, NULL);
}

/* As orc_rkck_solve, also recording the accepted step sizes (the first
 * rec_cap of them; *n_rec receives the count). */
int orc_rkck_solve_rec(const orc_problem *pb, const double *g, const double *y0, double *y1,
                       double t0, double t1, double rtol, double atol, int64_t max_steps,
                       int32_t *stats, double *rec_h, int64_t rec_cap, int64_t *n_rec) {
  int32_t *rs = rec_h && rec_cap > 0 ? (int32_t *)malloc(sizeof(int32_t) * (size_t)rec_cap) : NULL;
  step_rec r = {rec_h, rs, 0, rs ? rec_cap : 0, 0};
  int st = rkck_solve_impl(pb, g, y0, y1, t0, t1, rtol, atol, max_steps, stats, &r, NULL);
  if (n_rec) *n_rec = r.n;
  free(rs);
  return st;
}

/* ====================================================================== RKC */

/* RKC coefficients for s >= 2 stages (Sec. 2.2).  omega_0 = 1 + kappa/s^2 with
 * damping kappa = 2/13; T_j, T_j', T_j'' at omega_0 from the Chebyshev
 * recurrence T_j = 2x T_{j-1} - T_{j-2} and its first and second derivatives;
 * omega_1 = T_s'/T_s''; b_j = T_j''/(T_j')^2 (j >= 2); a_j = 1 - b_j T_j;
 * mut_1 = b_1 omega_1; mu_j = 2 b_j omega_0 / b_{j-1}; nu_j = -b_j / b_{j-2};
 * mut_j = 2 b_j omega_1 / b_{j-1}; gt_j = -a_{j-1} mut_j; c_1 = c_2 / T_2',
 * c_j = omega_1 T_j'' / T_j' (2 <= j <= s-1), c_s = 1.
 * Reading: b_0 = b_1 = b_2.  The printed b_1 = 1/omega_0 contradicts the
 * printed c_1 = c_2 / T_2'(omega_0): stage 1 sits at time mut_1 = b_1 omega_1,
 * and equating that with c_2 / T_2' = omega_1 / (4 omega_0^2) gives
 * b_1 = 1/(4 omega_0^2) = T_2''/(T_2')^2 = b_2.
 * All arrays have s + 1 entries (index j). */
int orc_rkc_coeffs(int s, double *w0p, double *w1p, double *T, double *D, double *E,
                   double *b, double *a, double *mu, double *nu, double *mut, double *gt,
                   double *c) {
  if (s < 2) return -1;
  const double kappa = 2.0 / 13.0;
  double w0 = 1.0 + kappa / ((double)s * (double)s);
  T[0] = 1.0;
  T[1] = w0;
  D[0] = 0.0;
  D[1] = 1.0;
  E[0] = 0.0;
  E[1] = 0.0;
  for (int j = 2; j <= s; ++j) {
    T[j] = 2.0 * w0 * T[j - 1] - T[j - 2];
    D[j] = 2.0 * T[j - 1] + 2.0 * w0 * D[j - 1] - D[j - 2];
    E[j] = 4.0 * D[j - 1] + 2.0 * w0 * E[j - 1] - E[j - 2];
  }
  double w1 = D[s] / E[s];
  for (int j = 2; j <= s; ++j) b[j] = E[j] / (D[j] * D[j]);
  b[0] = b[2];
  b[1] = b[2];
  for (int j = 0; j <= s; ++j) a[j] = 1.0 - b[j] * T[j];
  mu[0] = nu[0] = mut[0] = gt[0] = 0.0;
  mu[1] = nu[1] = gt[1] = 0.0;
  mut[1] = b[1] * w1;
  for (int j = 2; j <= s; ++j) {
    mu[j] = 2.0 * b[j] * w0 / b[j - 1];
    nu[j] = -b[j] / b[j - 2];
    mut[j] = 2.0 * b[j] * w1 / b[j - 1];
    gt[j] = -a[j - 1] * mut[j];
  }
  c[0] = 0.0;
  c[s] = 1.0;
  for (int j = 2; j <= s - 1; ++j) c[j] = w1 * E[j] / D[j];
  c[1] = c[2] / D[2];
  *w0p = w0;
  *w1p = w1;
  return 0;
}

typedef struct {
  int cap;
  double *T, *D, *E, *b, *a, *mu, *nu, *mut, *gt, *c;
  double w0, w1;
} rkc_tab;

static int tab_alloc(rkc_tab *tb, int cap) {
  tb->cap = cap;
  tb->T = (double *)malloc(sizeof(double) * 10 * (size_t)(cap + 1));
  if (!tb->T) return -2;
  tb->D = tb->T + (cap + 1);
  tb->E = tb->D + (cap + 1);
  tb->b = tb->E + (cap + 1);
  tb->a = tb->b + (cap + 1);
  tb->mu = tb->a + (cap + 1);
  tb->nu = tb->mu + (cap + 1);
  tb->mut = tb->nu + (cap + 1);
  tb->gt = tb->mut + (cap + 1);
  tb->c = tb->gt + (cap + 1);
  return 0;
}

static void tab_free(rkc_tab *tb) { free(tb->T); }

static void tab_fill(rkc_tab *tb, int s) {
  orc_rkc_coeffs(s, &tb->w0, &tb->w1, tb->T, tb->D, tb->E, tb->b, tb->a, tb->mu, tb->nu,
                 tb->mut, tb->gt, tb->c);
}

/* One RKC step with s stages (Eqs. E:rkc0 - E:rkcs): w_0 = y_n,
 * w_1 = w_0 + mut_1 h f_0, w_j = (1 - mu_j - nu_j) w_0 + mu_j w_{j-1}
 * + nu_j w_{j-2} + mut_j h f_{j-1} + gt_j h f_0, result w_s; f_0 = F is supplied.
 * If W is not NULL it receives every stage vector w_0..w_s ([s+1][N]). */
static void rkc_step(const orc_sys *S, const rkc_tab *tb, double t, const double *y,
                     const double *F, double h, int s, double *yout, double *W) {
  const int N = S->pb->n_eq;
  double wjm1[ORC_MAXN], wjm2[ORC_MAXN], wj[ORC_MAXN], f[ORC_MAXN];
  for (int i = 0; i < N; ++i) {
    wjm2[i] = y[i];
    wjm1[i] = y[i] + (tb->mut[1] * h) * F[i];
  }
  if (W) {
    memcpy(W, wjm2, sizeof(double) * N);
    memcpy(W + N, wjm1, sizeof(double) * N);
  }
  for (int j = 2; j <= s; ++j) {
    rhs(S, t + tb->c[j - 1] * h, wjm1, f);
    double c0 = 1.0 - tb->mu[j] - tb->nu[j];
    double mh = tb->mut[j] * h, gh = tb->gt[j] * h;
    for (int i = 0; i < N; ++i)
      wj[i] = c0 * y[i] + tb->mu[j] * wjm1[i] + tb->nu[j] * wjm2[i] + mh * f[i] + gh * F[i];
    for (int i = 0; i < N; ++i) {
      wjm2[i] = wjm1[i];
      wjm1[i] = wj[i];
    }
    if (W) memcpy(W + (size_t)j * N, wj, sizeof(double) * N);
  }
  for (int i = 0; i < N; ++i) yout[i] = wjm1[i];
}

int orc_rkc_step(const orc_problem *pb, const double *g, double t, const double *y,
                 const double *F, double h, int s, double *yout) {
  if (check_problem(pb) || s < 2) return -1;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  rkc_tab tb;
  if (!S || tab_alloc(&tb, s)) {
    free(S);
    return -2;
  }
  sys_init(S, pb, g);
  tab_fill(&tb, s);
  rkc_step(S, &tb, t, y, F, h, s, yout, NULL);
  tab_free(&tb);
  free(S);
  return 0;
}

/* All stage vectors w_0..w_s of one RKC step, [s+1][N]. */
int orc_rkc_stages(const orc_problem *pb, const double *g, double t, const double *y,
                   const double *F, double h, int s, double *W) {
  if (check_problem(pb) || s < 2) return -1;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  rkc_tab tb;
  double yout[ORC_MAXN];
  if (!S || tab_alloc(&tb, s)) {
    free(S);
    return -2;
  }
  sys_init(S, pb, g);
  tab_fill(&tb, s);
  rkc_step(S, &tb, t, y, F, h, s, yout, W);
  tab_free(&tb);
  free(S);
  return 0;
}

/* Nonlinear power method for the spectral radius of df/dy (Appendix): the
 * eigenvector estimate v is scaled to a perturbation of norm sqrt(UROUND)|y|
 * about y, and sigma = |f(v) - f(y)| / |v - y| is iterated, re-normalising the
 * difference each time, for at most itmax evaluations; the result is 1.2 sigma.
 * Reading: convergence is |sigma_k - sigma_{k-1}| <= 0.01 max(sigma_k, 1/hMax)
 * for k >= 2, the test of the method the appendix cites; the printed listing
 * overwrites the previous estimate with the relative change before comparing,
 * which would compare sigma with a number of order one and never converge.
 * On convergence v is returned as the direction v - y; otherwise it is left as
 * the last perturbed point, as printed.  F = f(t, y) is supplied. */
static double spec_rad(const orc_sys *S, double t, const double *y, const double *F,
                       double hmax, double *v, int itmax, int *iters) {
  const int N = S->pb->n_eq;
  double Fv[ORC_MAXN];
  const double sq = sqrt(UROUND);
  const double small = 1.0 / hmax;
  double ynrm = 0.0, vnrm = 0.0;
  for (int i = 0; i < N; ++i) {
    ynrm += y[i] * y[i];
    vnrm += v[i] * v[i];
  }
  ynrm = sqrt(ynrm);
  vnrm = sqrt(vnrm);
  double dynrm;
  if (ynrm != 0.0 && vnrm != 0.0) {
    dynrm = ynrm * sq;
    for (int i = 0; i < N; ++i) v[i] = y[i] + v[i] * (dynrm / vnrm);
  } else if (ynrm != 0.0) {
    dynrm = ynrm * sq;
    for (int i = 0; i < N; ++i) v[i] = y[i] * (1.0 + sq);
  } else if (vnrm != 0.0) {
    dynrm = UROUND;
    for (int i = 0; i < N; ++i) v[i] = v[i] * (dynrm / vnrm);
  } else {
    dynrm = UROUND;
    for (int i = 0; i < N; ++i) v[i] = UROUND;
  }
  double sigma = 0.0;
  for (int it = 1; it <= itmax; ++it) {
    rhs(S, t, v, Fv);
    double d = 0.0;
    for (int i = 0; i < N; ++i) d += (Fv[i] - F[i]) * (Fv[i] - F[i]);
    d = sqrt(d);
    double sprev = sigma;
    sigma = d / dynrm;
    if (it >= 2 && fabs(sigma - sprev) <= fmax(sigma, small) * 0.01) {
      for (int i = 0; i < N; ++i) v[i] = v[i] - y[i];
      *iters = it;
      return 1.2 * sigma;
    }
    if (d != 0.0) {
      for (int i = 0; i < N; ++i) v[i] = y[i] + (Fv[i] - F[i]) * (dynrm / d);
    } else {
      int ind = it % N;
      v[ind] = y[ind] - (v[ind] - y[ind]);
    }
  }
  *iters = itmax;
  return 1.2 * sigma;
}

double orc_spec_rad(const orc_problem *pb, const double *g, double t, const double *y,
                    const double *F, double hmax, double *v, int itmax, int *iters) {
  if (check_problem(pb)) return -1.0;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -1.0;
  sys_init(S, pb, g);
  double r = spec_rad(S, t, y, F, hmax, v, itmax, iters);
  free(S);
  return r;
}

/* Largest stage count (RKC driver listing): round(sqrt(rtol / (10 UROUND))),
 * at least 2 for second order. */
int orc_rkc_mmax(double rtol) {
  int m = (int)round(sqrt(rtol / (10.0 * UROUND)));
  return m < 2 ? 2 : m;
}

/* Stage count s = 1 + sqrt(1 + 1.54 h sigma) (Sec. 2.2), truncated to an
 * integer as in the driver listing; capped at mmax, in which case the step
 * is shortened to (s^2 - 1) / (1.54 sigma) so that it stays stable. */
int orc_rkc_stage_count(double h, double sigma, int mmax, double *h_out) {
  double x = sqrt(1.54 * h * sigma + 1.0);
  int m;
  if (x < (double)mmax) {
    m = 1 + (int)x;
  } else {
    m = mmax + 1; /* any value above the cap */
  }
  if (m > mmax) {
    m = mmax;
    h = ((double)m * (double)m - 1.0) / (1.54 * sigma);
  }
  *h_out = h;
  return m;
}

/* Step-size factor after an accepted RKC step (Eqs. dtnp1, rkc-f, in the form
 * of the driver listing): with a previous accepted step,
 * fac = min(10, 0.8 (h_n / h_{n-1}) err_{n-1}^{1/3} / err_n^{2/3}); for the
 * first accepted step fac = min(10, 0.8 / err^{1/3}).  The caller applies
 * max(0.1, fac).  Reading: the equation's indices are garbled; the listing's
 * ordering of terms is the one used. */
double orc_rkc_accept_factor(double err, double err_prev, double h, double h_prev,
                             int have_prev) {
  double fac = 10.0;
  if (!have_prev) {
    double t2 = orc_cr_pow(err, 1.0 / 3.0);
    if (0.8 < fac * t2) fac = 0.8 / t2;
  } else {
    double t1 = 0.8 * h * orc_cr_pow(err_prev, 1.0 / 3.0);
    double t2 = h_prev * orc_cr_pow(err, 2.0 / 3.0);
    if (t1 < fac * t2) fac = t1 / t2;
  }
  return fac;
}

/* ------------------------------------------------------- RKC controller parts
 * Each part of the RKC step-size and stage control of Sec. 2.2, as its own
 * function; the driver below combines them in the order of Sec. 3.2. */

/* Weighted RMS norm of Eq. E:rmsE: ||d / (T sqrt(N))||_2 with per-component
 * weights T = w, i.e. sqrt((1/N) sum_i (d_i / w_i)^2), squares summed in
 * index order. */
static double rms_norm(int n, const double *d, const double *w) {
  double e = 0.0;
  for (int i = 0; i < n; ++i) {
    const double q = d[i] / w[i];
    e += q * q;
  }
  return sqrt(e / (double)n);
}

/* A step size held within [hMin, hMax]. */
static double clamp_step(double h, double hmin, double hmax) {
  return fmax(hmin, fmin(hmax, h));
}

/* The step is stretched to reach t1 when t1 lies within 10% beyond it (the
 * driver of Sec. 3.2), so no sliver of a step is left at the end. */
static double stretch_to_end(double h, double t, double t1) {
  return (1.1 * h >= fabs(t1 - t)) ? fabs(t1 - t) : h;
}

/* Error of the step y_n -> y_{n+1} (Sec. 2.2):
 * Delta = 4/5 (y_n - y_{n+1}) + 2/5 h (f_n + f_{n+1}), measured by Eq. E:rmsE
 * with T = atol + rtol max(|y_n|, |y_{n+1}|). */
static double rkc_step_error(int n, const double *yn, const double *y, const double *Fn,
                             const double *F1, double h, double rtol, double atol) {
  double d[ORC_MAXN], w[ORC_MAXN];
  for (int i = 0; i < n; ++i) {
    d[i] = 0.8 * (yn[i] - y[i]) + 0.4 * h * (Fn[i] + F1[i]);
    w[i] = atol + rtol * fmax(fabs(y[i]), fabs(yn[i]));
  }
  return rms_norm(n, d, w);
}

/* Initial step size (Sec. 2.2).  A tentative forward-Euler step of size
 * dt0 = 1/sigma is taken from (t0, y0) with f0 = f(t0, y0); its error
 * Delta_0 = dt0 (f(t0 + dt0, y0 + dt0 f0) - f0) is measured by Eq. E:rmsE, and
 * the first step is dt1 = 0.1 dt0 / ||Delta_0||^(1/2).
 * Reading (the text does not bound dt0 or dt1; the driver of Sec. 3.2 does):
 * dt0 is hMax when sigma hMax <= 1 and at least hMin; dt1 is at least hMin and
 * is hMax whenever 0.1 dt0 >= hMax ||Delta_0||^(1/2) (the comparison is made
 * before dividing, so a zero error gives hMax).  The weights are
 * atol + rtol |y0| (the tentative state is not a solution value), and the norm
 * is that of f(...) - f0 times dt0, as the listing evaluates it. */
static double rkc_initial_step(const orc_sys *S, double t0, const double *y0, const double *f0,
                               double sigma, double hmin, double hmax, double rtol,
                               double atol) {
  const int N = S->pb->n_eq;
  double dt0 = hmax;
  if (sigma * dt0 > 1.0) dt0 = 1.0 / sigma;
  dt0 = fmax(dt0, hmin);
  double z[ORC_MAXN], f1[ORC_MAXN], d[ORC_MAXN], w[ORC_MAXN];
  for (int i = 0; i < N; ++i) z[i] = y0[i] + dt0 * f0[i];
  rhs(S, t0 + dt0, z, f1);
  for (int i = 0; i < N; ++i) {
    d[i] = f1[i] - f0[i];
    w[i] = atol + rtol * fabs(y0[i]);
  }
  const double err0 = dt0 * rms_norm(N, d, w);
  if (P1 * dt0 < hmax * sqrt(err0)) return fmax(P1 * dt0 / sqrt(err0), hmin);
  return hmax;
}

/* Step after a rejection (Eq. dtnp1 with f = 0.8 / err^(1/3), p = 2).
 * Reading: as in the driver of Sec. 3.2, without the equation's 0.1 floor (the
 * two differ only for err > 512).  A non-finite error (which the listing would
 * accept, NaN > 1 being false) cuts the step by P1, as the RKCK driver does. */
static double rkc_rejected_step(double err, double h) {
  return isfinite(err) ? 0.8 * h / orc_cr_pow(err, 1.0 / 3.0) : P1 * h;
}

/* Step after an accepted step: min(10, max(0.1, f)) h (Eq. dtnp1) with the
 * factor f of orc_rkc_accept_factor, then held within [hMin, hMax]. */
static double rkc_next_step(double err, double err_prev, double h, double h_prev, int have_prev,
                            double hmin, double hmax) {
  const double fac = orc_rkc_accept_factor(err, err_prev, h, h_prev, have_prev);
  return clamp_step(h * fmax(P1, fac), hmin, hmax);
}

/* Spectral radius of df/dy at (t, y_n) (Sec. 2.2, Appendix): the nonlinear
 * power method with the stored eigenvector estimate v, or the Gershgorin bound
 * of the analytic Jacobian when the problem asks for it.  Counts the call, its
 * iterations and their right-hand-side evaluations. */
static double rkc_sigma(const orc_sys *S, double t, const double *yn, const double *Fn,
                        double hmax, double *v, int64_t *n_sr, int64_t *n_pow, int64_t *n_rhs) {
  (*n_sr)++;
  if (S->pb->sr_method == 1) return gershgorin(S, yn, NULL);
  int it = 0;
  const double sigma = spec_rad(S, t, yn, Fn, hmax, v, 50, &it);
  *n_pow += it;
  *n_rhs += it;
  return sigma;
}

/* Accepted steps between refreshes of the spectral radius (Sec. 2.2: every
 * 25 internal steps, and after every rejected step). */
#define SR_PERIOD 25

/* RKC driver (Sec. 3.2, with the parts of Sec. 2.2 above).  Each attempt:
 * stretch the step to the end point if close; refresh sigma at the first step
 * and every SR_PERIOD accepted steps; on the first attempt choose the initial
 * step; pick the stage count (which may shorten the step); take the step and
 * evaluate f at its end; accept (advance, new step from Eq. dtnp1, f_{n+1}
 * becomes f_n) or reject (smaller step, sigma refreshed).
 * Reading (restart): every call starts fresh, with the previous-step memory
 * cleared and the eigenvector estimate v set to f(t0, y0); the listing's test
 * of a step size below UROUND as "not set yet" is replaced by explicit flags,
 * which agree with it whenever steps exceed UROUND.
 * Reading (refresh): the refresh at the loop top runs on every attempt made
 * while the accepted-step count is a multiple of SR_PERIOD, so a rejection at
 * such a count refreshes sigma twice (after the rejection and at the retry).
 * Guards as in the RKCK driver.  A trace, when given, receives one record per
 * attempt. */
static int rkc_solve_impl(const orc_problem *pb, const double *g, const double *y0, double *y1,
                          double t0, double t1, double rtol, double atol, int64_t max_steps,
                          int32_t *stats, step_rec *rec, double *carry, orc_rkc_attempt *trace,
                          int64_t trace_cap, int64_t *n_trace) {
  if (check_problem(pb) || !(t1 >= t0) || !(rtol > 0.0) || !(atol >= 0.0)) return -1;
  const int N = pb->n_eq;
  const int mmax = orc_rkc_mmax(rtol);
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  rkc_tab tb;
  if (!S || tab_alloc(&tb, mmax)) {
    free(S);
    return -2;
  }
  sys_init(S, pb, g);
  double y_n[ORC_MAXN], F_n[ORC_MAXN], y[ORC_MAXN], F1[ORC_MAXN], v[ORC_MAXN];
  const double hmax = fabs(t1 - t0);
  const double hmin = 10.0 * UROUND * fmax(fabs(t0), hmax);
  double t = t0;
  for (int i = 0; i < N; ++i) {
    y_n[i] = y0[i];
    F_n[i] = 0.0;
  }
  int64_t n_acc = 0, n_rej = 0, n_rhs = 0, n_sr = 0, n_pow = 0, attempts = 0, n_tr = 0;
  int max_m = 0, status = ORC_OK;
  if (t < t1) {
    rhs(S, t, y_n, F_n);
    n_rhs++;
  }
  for (int i = 0; i < N; ++i) v[i] = F_n[i];
  double h = 0.0, h_prev = 0.0, err_prev = 0.0, sigma = 0.0;
  int64_t nstep = 0;
  int first = 1, have_prev = 0, cut = 0;
  double h_want = 0.0;
  if (carry && carry[ORC_CARRY_VALID] != 0.0) {
    /* carried controller state (the alternative to the restart): the next
     * step, the previous step and error, the spectral radius and its
     * eigenvector, and the accepted-step count that schedules its refresh;
     * y_n and f(t0, y_n) are this call's */
    h = carry[ORC_CARRY_H];
    h_prev = carry[ORC_CARRY_H_PREV];
    err_prev = carry[ORC_CARRY_ERR_PREV];
    sigma = carry[ORC_CARRY_SIGMA];
    nstep = (int64_t)carry[ORC_CARRY_NSTEP];
    have_prev = carry[ORC_CARRY_HAVE_PREV] != 0.0;
    for (int i = 0; i < N; ++i) v[i] = carry[ORC_CARRY_ROWS + i];
    first = 0;
  }
  while (t < t1) {
    if (attempts >= max_steps) {
      status = ORC_MAXSTEPS;
      break;
    }
    h_want = h;
    h = stretch_to_end(h, t, t1);
    if (nstep % SR_PERIOD == 0) sigma = rkc_sigma(S, t, y_n, F_n, hmax, v, &n_sr, &n_pow, &n_rhs);
    if (first) {
      h = rkc_initial_step(S, t, y_n, F_n, sigma, hmin, hmax, rtol, atol);
      n_rhs++;
      first = 0;
    }
    const int m = orc_rkc_stage_count(h, sigma, mmax, &h);
    if (m > max_m) max_m = m;
    tab_fill(&tb, m);
    rkc_step(S, &tb, t, y_n, F_n, h, m, y, NULL);
    rhs(S, t + h, y, F1);
    n_rhs += m;
    const double err = rkc_step_error(N, y_n, y, F_n, F1, h, rtol, atol);
    attempts++;
    const int accept = err <= 1.0;   /* NaN and errors above 1 are rejected */
    if (trace && n_tr < trace_cap) {
      orc_rkc_attempt *a = trace + n_tr;
      a->t = t;
      a->h_want = h_want;
      a->h = h;
      a->sigma = sigma;
      a->err = err;
      a->m = m;
      a->accepted = accept;
      a->nstep = nstep;
      a->n_sr = n_sr;
    }
    n_tr++;
    if (!accept) {
      n_rej++;
      h = rkc_rejected_step(err, h);
      sigma = rkc_sigma(S, t, y_n, F_n, hmax, v, &n_sr, &n_pow, &n_rhs);
      if (!(h >= hmin)) {
        status = ORC_HMIN;
        break;
      }
    } else {
      cut = h < h_want;
      t += h;
      nstep++;
      n_acc++;
      rec_push(rec, h, m);
      const double hn = rkc_next_step(err, err_prev, h, h_prev, have_prev, hmin, hmax);
      err_prev = err;
      h_prev = h;
      have_prev = 1;
      for (int i = 0; i < N; ++i) {
        y_n[i] = y[i];
        F_n[i] = F1[i];
      }
      h = hn;
      if (!all_finite(N, y_n)) {
        status = ORC_NONFINITE;
        break;
      }
    }
  }
  if (n_trace) *n_trace = n_tr;
  if (carry) {
    carry[ORC_CARRY_VALID] = status == ORC_OK ? 1.0 : 0.0;
    carry[ORC_CARRY_H] = cut ? h_want : h;
    carry[ORC_CARRY_H_PREV] = h_prev;
    carry[ORC_CARRY_ERR_PREV] = err_prev;
    carry[ORC_CARRY_SIGMA] = sigma;
    carry[ORC_CARRY_NSTEP] = (double)nstep;
    carry[ORC_CARRY_HAVE_PREV] = have_prev ? 1.0 : 0.0;
    for (int i = 0; i < N; ++i) carry[ORC_CARRY_ROWS + i] = v[i];
  }
  for (int i = 0; i < N; ++i) y1[i] = y_n[i];
  if (stats) {
    stats[ORC_ST_ACCEPT] = (int32_t)n_acc;
    stats[ORC_ST_REJECT] = (int32_t)n_rej;
    stats[ORC_ST_RHS] = (int32_t)n_rhs;
    stats[ORC_ST_SR_CALLS] = (int32_t)n_sr;
    stats[ORC_ST_POW_ITERS] = (int32_t)n_pow;
    stats[ORC_ST_MAX_STAGES] = max_m;
  }
  tab_free(&tb);
  free(S);
  return status;
}

int orc_rkc_solve(const orc_problem *pb, const double *g, const double *y0, double *y1,
                  double t0, double t1, double rtol, double atol, int64_t max_steps,
                  int32_t *stats, double *rec_h, int32_t *rec_s, int64_t rec_cap,
                  int64_t *n_rec) {
  step_rec r = {rec_h, rec_s, 0, (rec_h && rec_s) ? rec_cap : 0, 0};
  int st = rkc_solve_impl(pb, g, y0, y1, t0, t1, rtol, atol, max_steps, stats, &r, NULL, NULL, 0,
                          NULL);
  if (n_rec) *n_rec = r.n;
  return st;
}

/* As orc_rkc_solve without the step record; trace (capacity trace_cap)
 * receives one record per attempt, *n_trace the number of attempts. */
int orc_rkc_solve_trace(const orc_problem *pb, const double *g, const double *y0, double *y1,
                        double t0, double t1, double rtol, double atol, int64_t max_steps,
                        int32_t *stats, orc_rkc_attempt *trace, int64_t trace_cap,
                        int64_t *n_trace) {
  return rkc_solve_impl(pb, g, y0, y1, t0, t1, rtol, atol, max_steps, stats, NULL, NULL, trace,
                        trace_cap, n_trace);
}

int orc_rkc_replay(const orc_problem *pb, const double *g, const double *y0, double t0,
                   int64_t n_steps, const double *h, const int32_t *s, double *y1) {
  if (check_problem(pb)) return -1;
  const int N = pb->n_eq;
  int smax = 2;
  for (int64_t k = 0; k < n_steps; ++k)
    if (s[k] > smax) smax = s[k];
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  rkc_tab tb;
  if (!S || tab_alloc(&tb, smax)) {
    free(S);
    return -2;
  }
  sys_init(S, pb, g);
  double y[ORC_MAXN], F[ORC_MAXN], yn[ORC_MAXN];
  for (int i = 0; i < N; ++i) y[i] = y0[i];
  double t = t0;
  for (int64_t k = 0; k < n_steps; ++k) {
    rhs(S, t, y, F);
    tab_fill(&tb, s[k]);
    rkc_step(S, &tb, t, y, F, h[k], s[k], yn, NULL);
    for (int i = 0; i < N; ++i) y[i] = yn[i];
    t += h[k];
  }
  for (int i = 0; i < N; ++i) y1[i] = y[i];
  tab_free(&tb);
  free(S);
  return 0;
}

/* Discrete adjoint of the accepted-step map with (h_k, s_k) held fixed:
 * for L = w . y(t1), lambda starts at w and is carried backwards through each
 * step by transposing the stage recursion of Eqs. E:rkc0 - E:rkcs:
 *   for j = s..2:  w0bar += (1 - mu_j - nu_j) wbar_j, wbar_{j-1} += mu_j wbar_j,
 *                  wbar_{j-2} += nu_j wbar_j, f0bar += gt_j h wbar_j,
 *                  u = mut_j h wbar_j: wbar_{j-1} += J(w_{j-1})^T u,
 *                  thetabar += (df/dtheta)(w_{j-1})^T u;
 *   then w0bar += wbar_1, f0bar += mut_1 h wbar_1, and f_0 = f(w_0) gives
 *   w0bar += J(w_0)^T f0bar, thetabar += (df/dtheta)(w_0)^T f0bar.
 * Every step-start state and every stage vector is stored (no checkpoints). */
int orc_rkc_replay_adjoint(const orc_problem *pb, const double *g, const double *y0,
                           double t0, int64_t n_steps, const double *h, const int32_t *s,
                           const double *w, double *dy0, double *dtheta) {
  if (check_vjp_problem(pb)) return -1;
  const int N = pb->n_eq;
  const int NT = orc_n_theta(pb);
  int smax = 2;
  for (int64_t k = 0; k < n_steps; ++k)
    if (s[k] > smax) smax = s[k];
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  double *Y = (double *)malloc(sizeof(double) * (size_t)(n_steps + 1) * N);
  double *Wst = (double *)malloc(sizeof(double) * (size_t)(smax + 1) * N);
  double *Wb = (double *)malloc(sizeof(double) * (size_t)(smax + 1) * N);
  double *tk = (double *)malloc(sizeof(double) * (size_t)(n_steps + 1));
  rkc_tab tb;
  int bad = (!S || !Y || !Wst || !Wb || !tk);
  if (bad || tab_alloc(&tb, smax)) {
    free(S); free(Y); free(Wst); free(Wb); free(tk);
    return -2;
  }
  sys_init(S, pb, g);
  double F[ORC_MAXN], yn[ORC_MAXN], lam[ORC_MAXN], f0b[ORC_MAXN], jtu[ORC_MAXN], u[ORC_MAXN];
  double th[ORC_MAXR + 1], thacc[ORC_MAXR + 1];
  /* forward replay, storing every step-start state */
  for (int i = 0; i < N; ++i) Y[i] = y0[i];
  tk[0] = t0;
  for (int64_t k = 0; k < n_steps; ++k) {
    const double *yk = Y + (size_t)k * N;
    rhs(S, tk[k], yk, F);
    tab_fill(&tb, s[k]);
    rkc_step(S, &tb, tk[k], yk, F, h[k], s[k], yn, NULL);
    for (int i = 0; i < N; ++i) Y[(size_t)(k + 1) * N + i] = yn[i];
    tk[k + 1] = tk[k] + h[k];
  }
  for (int i = 0; i < N; ++i) lam[i] = w[i];
  for (int j = 0; j < NT; ++j) thacc[j] = 0.0;
  for (int64_t k = n_steps - 1; k >= 0; --k) {
    const int sk = s[k];
    const double hk = h[k];
    const double *yk = Y + (size_t)k * N;
    rhs(S, tk[k], yk, F);
    tab_fill(&tb, sk);
    rkc_step(S, &tb, tk[k], yk, F, hk, sk, yn, Wst);
    for (size_t i = 0; i < (size_t)(sk + 1) * N; ++i) Wb[i] = 0.0;
    for (int i = 0; i < N; ++i) {
      Wb[(size_t)sk * N + i] = lam[i];
      f0b[i] = 0.0;
    }
    for (int j = sk; j >= 2; --j) {
      double *wbj = Wb + (size_t)j * N;
      double *wb1 = Wb + (size_t)(j - 1) * N;
      double *wb2 = Wb + (size_t)(j - 2) * N;
      double c0 = 1.0 - tb.mu[j] - tb.nu[j];
      for (int i = 0; i < N; ++i) {
        Wb[i] += c0 * wbj[i];
        wb1[i] += tb.mu[j] * wbj[i];
        wb2[i] += tb.nu[j] * wbj[i];
        f0b[i] += (tb.gt[j] * hk) * wbj[i];
        u[i] = (tb.mut[j] * hk) * wbj[i];
      }
      rhs_vjp(S, Wst + (size_t)(j - 1) * N, u, jtu, th);
      for (int i = 0; i < N; ++i) wb1[i] += jtu[i];
      for (int q = 0; q < NT; ++q) thacc[q] += th[q];
    }
    for (int i = 0; i < N; ++i) {
      Wb[i] += Wb[N + i];
      f0b[i] += (tb.mut[1] * hk) * Wb[N + i];
    }
    rhs_vjp(S, Wst, f0b, jtu, th);
    for (int i = 0; i < N; ++i) lam[i] = Wb[i] + jtu[i];
    for (int q = 0; q < NT; ++q) thacc[q] += th[q];
  }
  for (int i = 0; i < N; ++i) dy0[i] = lam[i];
  if (dtheta)
    for (int q = 0; q < NT; ++q) dtheta[q] = thacc[q];
  tab_free(&tb);
  free(S); free(Y); free(Wst); free(Wb); free(tk);
  return 0;
}

/* Replay of recorded RKCK steps: the fifth-order solution of each trial step
 * (Sec. 2.1) with the recorded step sizes, no error control. */
int orc_rkck_replay(const orc_problem *pb, const double *g, const double *y0, double t0,
                    int64_t n_steps, const double *h, double *y1) {
  if (check_problem(pb)) return -1;
  const int N = pb->n_eq;
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  if (!S) return -2;
  sys_init(S, pb, g);
  double y[ORC_MAXN], F[ORC_MAXN], yt[ORC_MAXN], ye[ORC_MAXN];
  for (int i = 0; i < N; ++i) y[i] = y0[i];
  double t = t0;
  for (int64_t k = 0; k < n_steps; ++k) {
    rhs(S, t, y, F);
    rkck_trial(S, t, y, F, h[k], yt, ye);
    for (int i = 0; i < N; ++i) y[i] = yt[i];
    t += h[k];
  }
  for (int i = 0; i < N; ++i) y1[i] = y[i];
  free(S);
  return 0;
}

/* Discrete adjoint of the RKCK accepted-step map with the step sizes held
 * fixed.  One step (Sec. 2.1 stage equations, Table 1 coefficients) is
 *   z_1 = y,  z_i = y + sum_{j<i} b_ij k_j,  k_i = h f(z_i),  y' = y + sum_i c_i k_i,
 * so for lambda = dL/dy' its transpose is
 *   kbar_i = c_i lambda,  ybar = lambda;  for i = 6..1:
 *     u = h kbar_i,  zbar = J(z_i)^T u,  thetabar += (df/dtheta)(z_i)^T u,
 *     ybar += zbar,  kbar_j += b_ij zbar (j < i);
 * and ybar is lambda for the step before.  Every step-start state is stored
 * and each step's stage states are recomputed (no checkpoints). */
int orc_rkck_replay_adjoint(const orc_problem *pb, const double *g, const double *y0,
                            double t0, int64_t n_steps, const double *h, const double *w,
                            double *dy0, double *dtheta) {
  if (check_vjp_problem(pb)) return -1;
  const int N = pb->n_eq;
  const int NT = orc_n_theta(pb);
  orc_sys *S = (orc_sys *)malloc(sizeof(orc_sys));
  double *Y = (double *)malloc(sizeof(double) * (size_t)(n_steps + 1) * N);
  double *tk = (double *)malloc(sizeof(double) * (size_t)(n_steps + 1));
  if (!S || !Y || !tk) {
    free(S); free(Y); free(tk);
    return -2;
  }
  sys_init(S, pb, g);
  double F[ORC_MAXN], yt[ORC_MAXN], ye[ORC_MAXN], Z[6 * ORC_MAXN];
  double lam[ORC_MAXN], yb[ORC_MAXN], kb[6][ORC_MAXN], u[ORC_MAXN], jtu[ORC_MAXN];
  double th[ORC_MAXR + 1], thacc[ORC_MAXR + 1];
  for (int i = 0; i < N; ++i) Y[i] = y0[i];
  tk[0] = t0;
  for (int64_t k = 0; k < n_steps; ++k) {
    const double *yk = Y + (size_t)k * N;
    rhs(S, tk[k], yk, F);
    rkck_trial(S, tk[k], yk, F, h[k], yt, ye);
    for (int i = 0; i < N; ++i) Y[(size_t)(k + 1) * N + i] = yt[i];
    tk[k + 1] = tk[k] + h[k];
  }
  for (int i = 0; i < N; ++i) lam[i] = w[i];
  for (int q = 0; q < NT; ++q) thacc[q] = 0.0;
  for (int64_t k = n_steps - 1; k >= 0; --k) {
    const double hk = h[k];
    const double *yk = Y + (size_t)k * N;
    rhs(S, tk[k], yk, F);
    rkck_trial_z(S, tk[k], yk, F, hk, yt, ye, Z);
    for (int st = 0; st < 6; ++st)
      for (int i = 0; i < N; ++i) kb[st][i] = RKCK_C[st] * lam[i];
    for (int i = 0; i < N; ++i) yb[i] = lam[i];
    for (int st = 5; st >= 0; --st) {
      for (int i = 0; i < N; ++i) u[i] = hk * kb[st][i];
      rhs_vjp(S, Z + (size_t)st * N, u, jtu, th);
      for (int q = 0; q < NT; ++q) thacc[q] += th[q];
      for (int i = 0; i < N; ++i) yb[i] += jtu[i];
      for (int j = 0; j < st; ++j)
        for (int i = 0; i < N; ++i) kb[j][i] += RKCK_B[st][j] * jtu[i];
    }
    for (int i = 0; i < N; ++i) lam[i] = yb[i];
  }
  for (int i = 0; i < N; ++i) dy0[i] = lam[i];
  if (dtheta)
    for (int q = 0; q < NT; ++q) dtheta[q] = thacc[q];
  free(S); free(Y); free(tk);
  return 0;
}

/* ------------------------------------------------------- complex step
 * Directional derivatives of the replayed step maps for the pins of the
 * adjoints: the same replay in complex arithmetic, started from
 * (y0 + i e dy0, theta + i e dtheta); the imaginary part of L over e is the
 * derivative along (dy0, dtheta) to within O(e^2), with no cancellation. */

#define CS_STEP 1.0e-20

typedef struct {
  const orc_sys *S;
  double complex kf[ORC_MAXR], kr[ORC_MAXR];
  double complex mu;
} cs_sys;

/* ln A_j + i e dtheta_j scales k_f,j and k_r,j by exp(i e dtheta_j). */
static void cs_init(cs_sys *Z, const orc_sys *S, const double *dtheta) {
  const orc_problem *pb = S->pb;
  Z->S = S;
  Z->mu = 0.0;
  if (pb->kind == ORC_VDP) Z->mu = S->g[0] + I * (CS_STEP * (dtheta ? dtheta[0] : 0.0));
  if (pb->kind == ORC_MASS_ACTION)
    for (int j = 0; j < pb->n_rx; ++j) {
      const double th = CS_STEP * (dtheta ? dtheta[j] : 0.0);
      const double complex e = cos(th) + I * sin(th);
      Z->kf[j] = S->kf[j] * e;
      Z->kr[j] = S->kr[j] * e;
    }
}

/* The right-hand side of rhs() in complex arithmetic. */
static void rhs_cs(const cs_sys *Z, const double complex *y, double complex *f) {
  const orc_problem *pb = Z->S->pb;
  const int N = pb->n_eq;
  if (pb->kind == ORC_VDP) {
    f[0] = y[1];
    f[1] = Z->mu * (1.0 - y[0] * y[0]) * y[1] - y[0];
  } else if (pb->kind == ORC_LINEAR) {
    for (int i = 0; i < N; ++i) {
      double complex s = 0.0;
      for (int j = 0; j < N; ++j) s += pb->A[i * N + j] * y[j];
      f[i] = s;
    }
  } else {
    double complex C[ORC_MAXN], omega[ORC_MAXN], M = 0.0;
    for (int k = 0; k < N; ++k) C[k] = (Z->S->rho * y[k]) * Z->S->invW[k];
    for (int k = 0; k < N; ++k) M += C[k];
    for (int k = 0; k < N; ++k) omega[k] = 0.0;
    for (int j = 0; j < pb->n_rx; ++j) {
      const int r0 = pb->reac[2 * j], r1 = pb->reac[2 * j + 1];
      const int p0 = pb->prod[2 * j], p1 = pb->prod[2 * j + 1];
      const double complex q = Z->kf[j] * C[r0] * (r1 >= 0 ? C[r1] : M) -
                               Z->kr[j] * C[p0] * (p1 >= 0 ? C[p1] : M);
      omega[r0] -= q;
      if (r1 >= 0) omega[r1] -= q;
      omega[p0] += q;
      if (p1 >= 0) omega[p1] += q;
    }
    for (int k = 0; k < N; ++k) f[k] = (pb->W[k] * omega[k]) * Z->S->irho;
  }
}

static int cs_setup(const orc_problem *pb, const double *g, const double *y0, const double *dy0,
                    const double *dtheta, orc_sys **S, cs_sys **Z, double complex *y) {
  if (check_vjp_problem(pb)) return -1;
  *S = (orc_sys *)malloc(sizeof(orc_sys));
  *Z = (cs_sys *)malloc(sizeof(cs_sys));
  if (!*S || !*Z) {
    free(*S);
    free(*Z);
    return -2;
  }
  sys_init(*S, pb, g);
  cs_init(*Z, *S, dtheta);
  for (int i = 0; i < pb->n_eq; ++i) y[i] = y0[i] + I * (CS_STEP * (dy0 ? dy0[i] : 0.0));
  return 0;
}

static double cs_result(int n, const double *w, const double complex *y) {
  double complex L = 0.0;
  for (int i = 0; i < n; ++i) L += w[i] * y[i];
  return cimag(L) / CS_STEP;
}

int orc_rkc_replay_jvp_cs(const orc_problem *pb, const double *g, const double *y0, double t0,
                          int64_t n_steps, const double *h, const int32_t *s, const double *w,
                          const double *dy0, const double *dtheta, double *jvp) {
  (void)t0;
  orc_sys *S;
  cs_sys *Z;
  double complex y[ORC_MAXN], F[ORC_MAXN], f[ORC_MAXN], wjm1[ORC_MAXN], wjm2[ORC_MAXN],
      wj[ORC_MAXN];
  int rc = cs_setup(pb, g, y0, dy0, dtheta, &S, &Z, y);
  if (rc) return rc;
  const int N = pb->n_eq;
  int smax = 2;
  for (int64_t k = 0; k < n_steps; ++k)
    if (s[k] > smax) smax = s[k];
  rkc_tab tb;
  if (tab_alloc(&tb, smax)) {
    free(S);
    free(Z);
    return -2;
  }
  for (int64_t k = 0; k < n_steps; ++k) {
    const double hk = h[k];
    tab_fill(&tb, s[k]);
    rhs_cs(Z, y, F);
    for (int i = 0; i < N; ++i) {
      wjm2[i] = y[i];
      wjm1[i] = y[i] + (tb.mut[1] * hk) * F[i];
    }
    for (int j = 2; j <= s[k]; ++j) {
      rhs_cs(Z, wjm1, f);
      const double c0 = 1.0 - tb.mu[j] - tb.nu[j];
      for (int i = 0; i < N; ++i)
        wj[i] = c0 * y[i] + tb.mu[j] * wjm1[i] + tb.nu[j] * wjm2[i] + (tb.mut[j] * hk) * f[i] +
                (tb.gt[j] * hk) * F[i];
      for (int i = 0; i < N; ++i) {
        wjm2[i] = wjm1[i];
        wjm1[i] = wj[i];
      }
    }
    for (int i = 0; i < N; ++i) y[i] = wjm1[i];
  }
  *jvp = cs_result(N, w, y);
  tab_free(&tb);
  free(S);
  free(Z);
  return 0;
}

int orc_rkck_replay_jvp_cs(const orc_problem *pb, const double *g, const double *y0, double t0,
                           int64_t n_steps, const double *h, const double *w, const double *dy0,
                           const double *dtheta, double *jvp) {
  (void)t0;
  orc_sys *S;
  cs_sys *Z;
  double complex y[ORC_MAXN], z[ORC_MAXN], k[6][ORC_MAXN], f[ORC_MAXN];
  int rc = cs_setup(pb, g, y0, dy0, dtheta, &S, &Z, y);
  if (rc) return rc;
  const int N = pb->n_eq;
  for (int64_t n = 0; n < n_steps; ++n) {
    const double hk = h[n];
    rhs_cs(Z, y, f);
    for (int i = 0; i < N; ++i) k[0][i] = hk * f[i];
    for (int st = 1; st < 6; ++st) {
      for (int i = 0; i < N; ++i) {
        double complex acc = y[i];
        for (int j = 0; j < st; ++j) acc = acc + RKCK_B[st][j] * k[j][i];
        z[i] = acc;
      }
      rhs_cs(Z, z, f);
      for (int i = 0; i < N; ++i) k[st][i] = hk * f[i];
    }
    for (int i = 0; i < N; ++i) {
      double complex acc = y[i];
      for (int st = 0; st < 6; ++st) acc = acc + RKCK_C[st] * k[st][i];
      y[i] = acc;
    }
  }
  *jvp = cs_result(N, w, y);
  free(S);
  free(Z);
  return 0;
}

/* ------------------------------------------------------------------ batches */

int orc_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static void gather(const double *soa, int64_t n, int64_t i, int rows, double *out) {
  for (int r = 0; r < rows; ++r) out[r] = soa[(size_t)r * n + i];
}

static void scatter(double *soa, int64_t n, int64_t i, int rows, const double *in) {
  for (int r = 0; r < rows; ++r) soa[(size_t)r * n + i] = in[r];
}

static int batch_common(int method, const orc_problem *pb, int64_t n, const double *y0,
                        const double *g, double *y1, double t0, double t1, double rtol,
                        double atol, int64_t max_steps, int32_t *status, int32_t *stats,
                        double *carry, int n_threads) {
  if (check_problem(pb) || n < 0 || !(t1 >= t0) || !(rtol > 0.0) || !(atol >= 0.0)) return -1;
  const int N = pb->n_eq, P = pb->n_param;
  int nt = n_threads > 0 ? n_threads : orc_max_threads();
  int failed = 0;
  (void)nt;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nt)
  for (int64_t i = 0; i < n; ++i) {
    double ys[ORC_MAXN], yo[ORC_MAXN], gs[ORC_MAXP], cs[ORC_CARRY_ROWS + ORC_MAXN];
    int32_t st[ORC_NSTATS];
    gather(y0, n, i, N, ys);
    gather(g, n, i, P, gs);
    if (carry) gather(carry, n, i, ORC_CARRY_ROWS + N, cs);
    double *cp = carry ? cs : NULL;
    int rc = (method == 0)
                 ? rkck_solve_impl(pb, gs, ys, yo, t0, t1, rtol, atol, max_steps, st, NULL, cp)
                 : rkc_solve_impl(pb, gs, ys, yo, t0, t1, rtol, atol, max_steps, st, NULL, cp, NULL,
                                  0, NULL);
    if (rc < 0) {
#pragma omp atomic write
      failed = 1;
      continue;
    }
    scatter(y1, n, i, N, yo);
    if (carry) scatter(carry, n, i, ORC_CARRY_ROWS + N, cs);
    if (status) status[i] = rc;
    if (stats)
      for (int r = 0; r < ORC_NSTATS; ++r) stats[(size_t)r * n + i] = st[r];
  }
  return failed ? -2 : 0;
}

int orc_rkck_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                   double *y1, double t0, double t1, double rtol, double atol,
                   int64_t max_steps, int32_t *status, int32_t *stats, int n_threads) {
  return batch_common(0, pb, n, y0, g, y1, t0, t1, rtol, atol, max_steps, status, stats, NULL,
                      n_threads);
}

int orc_rkc_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                  double *y1, double t0, double t1, double rtol, double atol,
                  int64_t max_steps, int32_t *status, int32_t *stats, int n_threads) {
  return batch_common(1, pb, n, y0, g, y1, t0, t1, rtol, atol, max_steps, status, stats, NULL,
                      n_threads);
}

int orc_rkc_adjoint_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                          double t0, double t1, double rtol, double atol, int64_t max_steps,
                          const double *w, double *y1, double *dy0, double *dtheta,
                          int32_t *status, int n_threads) {
  if (check_vjp_problem(pb) || n < 0 || !(t1 >= t0) || !(rtol > 0.0) || !(atol >= 0.0)) return -1;
  const int N = pb->n_eq, P = pb->n_param, NT = orc_n_theta(pb);
  int nt = n_threads > 0 ? n_threads : orc_max_threads();
  int failed = 0;
  (void)nt;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
  for (int64_t i = 0; i < n; ++i) {
    double ys[ORC_MAXN], yo[ORC_MAXN], gs[ORC_MAXP], ws[ORC_MAXN], d0[ORC_MAXN];
    double dth[ORC_MAXR + 1];
    gather(y0, n, i, N, ys);
    gather(g, n, i, P, gs);
    gather(w, n, i, N, ws);
    step_rec r = {NULL, NULL, 0, 0, 1};
    int rc = rkc_solve_impl(pb, gs, ys, yo, t0, t1, rtol, atol, max_steps, NULL, &r, NULL, NULL,
                            0, NULL);
    int rc2 = (rc >= 0 && r.n <= r.cap)
                  ? orc_rkc_replay_adjoint(pb, gs, ys, t0, r.n, r.h, r.s, ws, d0, dth)
                  : -2;
    free(r.h);
    free(r.s);
    if (rc < 0 || rc2 < 0) {
#pragma omp atomic write
      failed = 1;
      continue;
    }
    scatter(y1, n, i, N, yo);
    scatter(dy0, n, i, N, d0);
    if (dtheta) scatter(dtheta, n, i, NT, dth);
    if (status) status[i] = rc;
  }
  return failed ? -2 : 0;
}

int orc_rkck_adjoint_batch(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                           double t0, double t1, double rtol, double atol, int64_t max_steps,
                           const double *w, double *y1, double *dy0, double *dtheta,
                           int32_t *status, int n_threads) {
  if (check_vjp_problem(pb) || n < 0 || !(t1 >= t0) || !(rtol > 0.0) || !(atol >= 0.0)) return -1;
  const int N = pb->n_eq, P = pb->n_param, NT = orc_n_theta(pb);
  int nt = n_threads > 0 ? n_threads : orc_max_threads();
  int failed = 0;
  (void)nt;
#pragma omp parallel for schedule(dynamic, 4) num_threads(nt)
  for (int64_t i = 0; i < n; ++i) {
    double ys[ORC_MAXN], yo[ORC_MAXN], gs[ORC_MAXP], ws[ORC_MAXN], d0[ORC_MAXN];
    double dth[ORC_MAXR + 1];
    gather(y0, n, i, N, ys);
    gather(g, n, i, P, gs);
    gather(w, n, i, N, ws);
    step_rec r = {NULL, NULL, 0, 0, 1};
    int rc = rkck_solve_impl(pb, gs, ys, yo, t0, t1, rtol, atol, max_steps, NULL, &r, NULL);
    int rc2 = (rc >= 0 && r.n <= r.cap)
                  ? orc_rkck_replay_adjoint(pb, gs, ys, t0, r.n, r.h, ws, d0, dth)
                  : -2;
    free(r.h);
    free(r.s);
    if (rc < 0 || rc2 < 0) {
#pragma omp atomic write
      failed = 1;
      continue;
    }
    scatter(y1, n, i, N, yo);
    scatter(dy0, n, i, N, d0);
    if (dtheta) scatter(dtheta, n, i, NT, dth);
    if (status) status[i] = rc;
  }
  return failed ? -2 : 0;
}

/* Batches with the controller state carried between calls: carry [rows][n]
 * SoA, rows ORC_CARRY_ROWS + N (RKCK uses the first two), updated in place. */
int orc_rkck_batch_carry(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                         double *y1, double t0, double t1, double rtol, double atol,
                         int64_t max_steps, int32_t *status, int32_t *stats, double *carry,
                         int n_threads) {
  return batch_common(0, pb, n, y0, g, y1, t0, t1, rtol, atol, max_steps, status, stats, carry,
                      n_threads);
}

int orc_rkc_batch_carry(const orc_problem *pb, int64_t n, const double *y0, const double *g,
                        double *y1, double t0, double t1, double rtol, double atol,
                        int64_t max_steps, int32_t *status, int32_t *stats, double *carry,
                        int n_threads) {
  return batch_common(1, pb, n, y0, g, y1, t0, t1, rtol, atol, max_steps, status, stats, carry,
                      n_threads);
}
