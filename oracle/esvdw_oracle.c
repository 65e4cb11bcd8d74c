/*
 * esvdw_oracle.c -- plain, slow, FP64 CPU reference of the adaptive moving-mesh
 * entropy-stable finite-difference scheme for the Euler equations with the
 * van der Waals equation of state (Li & Tang, arXiv 2407.05568).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark may load this file's library.  It shares no source with the GPU
 * library and is written for readability, not speed: explicit ghost-padded arrays,
 * explicit matrices, scalar loops, no fusion.  Build with -O2 -ffp-contract=off.
 *
 * Units: general (R, c_v, a, b); the flux pressure is p itself.  The paper's own
 * dimensionless units are (R, c_v, a, b) = (1, 1/delta, 9/8, 1/3), where p equals
 * 3/8 of the dimensionless p_* (Section 2).
 *
 * Readings where the paper is silent:
 *  - nodes are cell-centred, xi_i = lo + (i + 1/2) dxi;
 *  - ghost states copy the nearest interior node (outflow) or wrap (periodic);
 *    ghost mesh nodes mirror about the boundary face (normal coordinate odd,
 *    tangential even) or wrap with a shift of one period;
 *  - the interface eigen-system uses arithmetic means of the node metrics;
 *  - the multi-resolution WENO (only cited by the paper) is the three-level
 *    1/3/5-point hierarchy with the tau-based nonlinear weights in mrweno5();
 *  - the stage mesh of SSP-RK3 is x^n + c_s dt xdot with c = (0, 1, 1/2);
 *  - the CFL spectral radius excludes the mesh velocity and divides by J.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NVMAX 5
#define GS 3  /* ghost width of node states and metrics */
#define GM 6  /* ghost width of the mesh (metrics are needed at 3 ghost nodes) */

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1 };
enum { F_INADMISSIBLE = 1u, F_MEANCONSTRAINT = 2u, F_NAN = 4u, F_NOTCONVERGED = 8u };
enum { MON_VDW = 0, MON_SINE = 1 };
enum { VAR_RHO = 0, VAR_G = 1 };

typedef struct {
  int dim;
  int n[3];
  double lo[3], hi[3];
  int bc[3];
  double R, cv, a, b;
  int dissipation;          /* 0: entropy conservative only, 1: entropy stable */
  double weno_lin[3];       /* linear weights of the 5-, 3- and 1-point levels */
  double weno_eps;
  double cfl;
  double dt_fixed;          /* > 0: use this time step instead of the CFL one */
  int monitor_kind;         /* MON_VDW or MON_SINE */
  int kappa;                /* number of gradient terms in the vdW monitor */
  int mon_var[2];           /* VAR_RHO or VAR_G for each gradient term */
  double alpha[3];          /* alpha_1 .. alpha_{kappa+1} */
  int n_filter;
  int mu;                   /* Jacobi sweeps (fixed), or the cap in tolerance mode */
  double mesh_tol;
  int fixed_mu;             /* 1: exactly mu sweeps; 0: stop when the update < tol */
  int walls;                /* bit 2k: the lo face of direction k is a reflecting wall; 2k+1: hi */
  /* 2D backward-facing step (Example 5.5): the nodes i0 < step[0], i1 < step[1] are solid, the
     fluid is the L-shaped rest; both faces of the step are reflecting walls.  0: no step. */
  int step[2];
  int inflow;               /* 1: the lo face of direction 0 holds the fixed state inflow_prim */
  double inflow_prim[4];    /* rho, v_1, v_2, p */
} orc_cfg;

static unsigned g_flags = 0;

/* flags are raised from the parallel loops of the OpenMP build: atomically there */
static void raise_flag(unsigned f) {
#pragma omp atomic
  g_flags |= f;
}

/* threads of the OpenMP build (the CPU baseline); 1 in the plain build */
int orc_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
  return omp_get_max_threads();
#else
  (void)n;
  return 1;
#endif
}

unsigned orc_get_flags(int clear) {
  unsigned f = g_flags;
  if (clear) g_flags = 0;
  return f;
}

/* ------------------------------------------------------------------------- */
/* Equation of state (eq. vdWEOS, Section 1; dimensionless forms Section 2)   */
/* ------------------------------------------------------------------------- */

static double eos_pressure(const orc_cfg *c, double rho, double T) {
  return rho * c->R * T / (1.0 - c->b * rho) - c->a * rho * rho;
}

static double eos_energy(const orc_cfg *c, double rho, double T) {
  return c->cv * T - c->a * rho;
}

double orc_T_from_rho_p(const orc_cfg *c, double rho, double p) {
  /* invert p = rho R T/(1 - b rho) - a rho^2 for T */
  return (p + c->a * rho * rho) * (1.0 - c->b * rho) / (rho * c->R);
}

static double eos_sound2(const orc_cfg *c, double rho, double T) {
  double delta = c->R / c->cv;
  double ob = 1.0 - c->b * rho;
  return (delta + 1.0) * c->R * T / (ob * ob) - 2.0 * c->a * rho;
}

/* fundamental derivative G = nu^3/(2 c^2) (d^2 p / d nu^2)_s in closed form
   (eq. fundamental; Section 2 gives the dimensionless version) */
static double eos_G(const orc_cfg *c, double rho, double T) {
  double delta = c->R / c->cv;
  double ob = 1.0 - c->b * rho;
  double c2 = eos_sound2(c, rho, T);
  return ((delta + 1.0) * (delta + 2.0) * c->R * T / (ob * ob * ob) - 6.0 * c->a * rho) / (2.0 * c2);
}

/* specific entropy s = c_v ln T + R ln(nu - b) (the sign of the second term in
   the Introduction is a typo: the dimensionless s_* of Section 2 and the entropy
   variables fix it as +) */
static double eos_entropy(const orc_cfg *c, double rho, double T) {
  return c->cv * log(T) + c->R * log(1.0 / rho - c->b);
}

/* admissible states, eq. coefflimit and eq. Tlimit */
int orc_admissible(const orc_cfg *c, double rho, double T) {
  if (!(rho > 0.0)) return 0;
  if (c->b > 0.0 && !(rho < 1.0 / c->b)) return 0;
  if (c->b > 0.0) {
    if (!(T > c->a / (4.0 * c->R * c->b))) return 0;
  } else if (!(T > 0.0)) return 0;
  double ob = 1.0 - c->b * rho;
  if (!(c->R * T - 2.0 * c->a * rho * ob * ob > 0.0)) return 0;
  return 1;
}

/* out = {p, e, c^2, G, s} */
void orc_eos_state(const orc_cfg *c, double rho, double T, double *out) {
  out[0] = eos_pressure(c, rho, T);
  out[1] = eos_energy(c, rho, T);
  out[2] = eos_sound2(c, rho, T);
  out[3] = eos_G(c, rho, T);
  out[4] = eos_entropy(c, rho, T);
}

/* ------------------------------------------------------------------------- */
/* Conserved / primitive variables, entropy pair (Section 2)                  */
/* ------------------------------------------------------------------------- */

/* prim = (rho, v_1..v_d, p) -> U = (rho, rho v, E) */
void orc_prim_to_cons(const orc_cfg *c, const double *prim, double *U) {
  int d = c->dim;
  double rho = prim[0], p = prim[d + 1];
  double T = orc_T_from_rho_p(c, rho, p);
  double v2 = 0.0;
  U[0] = rho;
  for (int m = 0; m < d; ++m) {
    U[1 + m] = rho * prim[1 + m];
    v2 += prim[1 + m] * prim[1 + m];
  }
  U[d + 1] = rho * eos_energy(c, rho, T) + 0.5 * rho * v2;
}

/* U -> z = (rho, v_1..v_d, T) (the parameter vector, eq. parameter_vector) */
static void cons_to_z(const orc_cfg *c, const double *U, double *z) {
  int d = c->dim;
  double rho = U[0], v2 = 0.0;
  z[0] = rho;
  for (int m = 0; m < d; ++m) {
    z[1 + m] = U[1 + m] / rho;
    v2 += z[1 + m] * z[1 + m];
  }
  double e = U[d + 1] / rho - 0.5 * v2;
  z[d + 1] = (e + c->a * rho) / c->cv;
  if (!orc_admissible(c, rho, z[d + 1])) raise_flag(F_INADMISSIBLE);
  if (isnan(rho) || isnan(z[d + 1])) raise_flag(F_NAN);
}

/* prim = (rho, v, p, T) from U, exported for tests */
void orc_cons_to_prim(const orc_cfg *c, const double *U, double *prim) {
  double z[NVMAX];
  int d = c->dim;
  cons_to_z(c, U, z);
  for (int m = 0; m <= d; ++m) prim[m] = z[m];
  prim[d + 1] = eos_pressure(c, z[0], z[d + 1]);
  prim[d + 2] = z[d + 1];
}

/* entropy eta = -rho s (eq. van der WaalsEntropy) */
double orc_entropy(const orc_cfg *c, const double *U) {
  double z[NVMAX];
  cons_to_z(c, U, z);
  return -z[0] * eos_entropy(c, z[0], z[c->dim + 1]);
}

/* entropy variables V = eta'(U) */
void orc_entropy_vars(const orc_cfg *c, const double *U, double *V) {
  int d = c->dim;
  double z[NVMAX];
  cons_to_z(c, U, z);
  double rho = z[0], T = z[d + 1], v2 = 0.0;
  for (int m = 0; m < d; ++m) v2 += z[1 + m] * z[1 + m];
  double e = eos_energy(c, rho, T), p = eos_pressure(c, rho, T);
  V[0] = -eos_entropy(c, rho, T) + (e + p / rho - 0.5 * v2) / T;
  for (int m = 0; m < d; ++m) V[1 + m] = z[1 + m] / T;
  V[d + 1] = -1.0 / T;
}

/* entropy potential phi = V.U - eta and flux potentials psi_k = V.F_k - q_k,
   evaluated from their definitions */
void orc_potentials(const orc_cfg *c, const double *U, double *phi, double *psi);

/* physical flux F_j(U) in direction j (eq. ConserLaw3) */
void orc_phys_flux(const orc_cfg *c, const double *U, int j, double *F) {
  int d = c->dim;
  double z[NVMAX];
  cons_to_z(c, U, z);
  double rho = z[0], vj = z[1 + j], p = eos_pressure(c, rho, z[d + 1]);
  F[0] = rho * vj;
  for (int m = 0; m < d; ++m) F[1 + m] = rho * vj * z[1 + m] + (m == j ? p : 0.0);
  F[d + 1] = (U[d + 1] + p) * vj;
}

void orc_potentials(const orc_cfg *c, const double *U, double *phi, double *psi) {
  int d = c->dim, nv = d + 2;
  double V[NVMAX], F[NVMAX], z[NVMAX];
  orc_entropy_vars(c, U, V);
  cons_to_z(c, U, z);
  double eta = orc_entropy(c, U);
  double acc = 0.0;
  for (int i = 0; i < nv; ++i) acc += V[i] * U[i];
  *phi = acc - eta;
  for (int j = 0; j < d; ++j) {
    orc_phys_flux(c, U, j, F);
    acc = 0.0;
    for (int i = 0; i < nv; ++i) acc += V[i] * F[i];
    psi[j] = acc - eta * z[1 + j];  /* q_j = -rho s v_j = eta v_j */
  }
}

/* ------------------------------------------------------------------------- */
/* Logarithmic mean (Ismail-Roe), used in Section 3.1 and Section 3.3         */
/* ------------------------------------------------------------------------- */

/* L(al, ar) = (ar - al)/(ln ar - ln al), evaluated as (al + ar)/(2 atanh(f)/f)
   with f = (ar - al)/(ar + al); a five-term series of atanh(f)/f for f^2 < 1e-4
   keeps full precision when al and ar are close. */
double orc_logmean(double al, double ar) {
  double f = (ar - al) / (ar + al);
  double u = f * f;
  double F;
  if (u < 1e-4)
    F = 1.0 + u / 3.0 + u * u / 5.0 + u * u * u / 7.0 + u * u * u * u / 9.0;
  else
    F = 0.5 * log1p(2.0 * f / (1.0 - f)) / f;
  return (al + ar) / (2.0 * F);
}

/* ------------------------------------------------------------------------- */
/* Two-point entropy-conservative flux (Section 3.1, eq. ECCondition_comp)    */
/* ------------------------------------------------------------------------- */

/* Solves the linear systems eq. linear_U / eq. linear_F in closed form, for general
 * (R, c_v, a, b) and d velocity components.  With the parameter vector z = (rho, v, T):
 *   [V_1] = D [rho] + (-c_v/L(T) + 2a{rho/T}/{T} + 1/2 sum {v_m^2/T}/{T}) [T] - sum {v_m}[v_m]/{T}
 *   [V_{1+m}] = [v_m]/{T} - {v_m/T}[T]/{T},   [V_E] = {1/T}[T]/{T}
 *   D = R/L(rho) + R b/L(1 - b rho) + R b/((1 - b rho_l)(1 - b rho_r)) - 2a/{T}
 *   [phi] = [rho g], [psi_j] = [rho v_j g],  g = R/(1 - b rho) - a rho/T  (phi = p/T)
 * Matching the coefficients of [rho], [v_m], [T] gives Ut and Ft below.  In the paper's
 * units this reproduces the printed U~ and F~_1 term by term; D is the quantity whose
 * positivity Theorem 3.1 establishes.
 * Ut[nv], Ft[j*NVMAX + i] for j < d. */
void orc_ec_pair(const orc_cfg *c, const double *Ul, const double *Ur, double *Ut, double *Ft) {
  int d = c->dim;
  double zl[NVMAX], zr[NVMAX];
  cons_to_z(c, Ul, zl);
  cons_to_z(c, Ur, zr);
  double R = c->R, cv = c->cv, a = c->a, b = c->b;
  double rl = zl[0], rr = zr[0], Tl = zl[d + 1], Tr = zr[d + 1];
  /* arithmetic means {.} */
  double m_rho = 0.5 * (rl + rr);
  double m_T = 0.5 * (Tl + Tr);
  double m_invT = 0.5 * (1.0 / Tl + 1.0 / Tr);
  double m_rhoT = 0.5 * (rl / Tl + rr / Tr);
  double gl = R / (1.0 - b * rl) - a * rl / Tl;
  double gr = R / (1.0 - b * rr) - a * rr / Tr;
  double m_g = 0.5 * (gl + gr);
  double m_v[3], m_vT[3], m_v2T = 0.0, m_rhov[3];
  for (int m = 0; m < d; ++m) {
    m_v[m] = 0.5 * (zl[1 + m] + zr[1 + m]);
    m_vT[m] = 0.5 * (zl[1 + m] / Tl + zr[1 + m] / Tr);
    m_v2T += 0.5 * (zl[1 + m] * zl[1 + m] / Tl + zr[1 + m] * zr[1 + m] / Tr);
    m_rhov[m] = 0.5 * (rl * zl[1 + m] + rr * zr[1 + m]);
  }
  double Pi = (1.0 - b * rl) * (1.0 - b * rr);
  double D = R / orc_logmean(rl, rr) - 2.0 * a / m_T + R * b / Pi;
  if (b > 0.0) D += R * b / orc_logmean(1.0 - b * rl, 1.0 - b * rr);
  double A = R * b / Pi - a / m_T;
  double K = 0.5 * m_v2T - cv * m_T / orc_logmean(Tl, Tr) + 2.0 * a * m_rhoT;
  /* Theorem 3.1: the system is uniquely solvable when the mean state satisfies
     R{T} - 2a{rho}(1 - b{rho})^2 > 0 (eq. mean_constraint); then D > 0 */
  double obm = 1.0 - b * m_rho;
  if (!(D > 0.0) || !(R * m_T - 2.0 * a * m_rho * obm * obm > 0.0)) raise_flag(F_MEANCONSTRAINT);

  /* U~ */
  Ut[0] = (m_rho * A + m_g) / D;
  for (int m = 0; m < d; ++m) Ut[1 + m] = m_v[m] * Ut[0];
  {
    double s = 0.0;
    for (int m = 0; m < d; ++m) s += m_vT[m] * Ut[1 + m];
    Ut[d + 1] = (s - K * Ut[0] + a * m_rho * m_rhoT) / m_invT;
  }
  /* F~_j */
  for (int j = 0; j < d; ++j) {
    double *F = Ft + j * NVMAX;
    F[0] = (m_rhov[j] * A + m_g * m_v[j]) / D;
    for (int m = 0; m < d; ++m) F[1 + m] = m_v[m] * F[0] + (m == j ? m_rho * m_T * m_g : 0.0);
    double s = 0.0;
    for (int m = 0; m < d; ++m) s += m_vT[m] * F[1 + m];
    F[d + 1] = (s - K * F[0] + a * m_rhov[j] * m_rhoT) / m_invT;
  }
}

/* curvilinear two-point flux (eq. ECfluxMM): {J xi_k/t} U~ + sum_j {J xi_k/x_j} F~_j.
   mtl, mtr: J xi_k/t of the two nodes; mxl[j], mxr[j]: J xi_k/x_j. */
static void ec_pair_curv(const orc_cfg *c, const double *Ul, const double *Ur,
                         double mtl, double mtr, const double *mxl, const double *mxr, double *Fh) {
  int d = c->dim, nv = d + 2;
  double Ut[NVMAX], Ft[3 * NVMAX];
  orc_ec_pair(c, Ul, Ur, Ut, Ft);
  for (int i = 0; i < nv; ++i) {
    double v = 0.5 * (mtl + mtr) * Ut[i];
    for (int j = 0; j < d; ++j) v += 0.5 * (mxl[j] + mxr[j]) * Ft[j * NVMAX + i];
    Fh[i] = v;
  }
}

/* alpha_{w,m} for w = 3 from sum m alpha = 1, sum m^3 alpha = sum m^5 alpha = 0 */
static const double ALPHA[3] = {1.5, -0.3, 1.0 / 30.0};

void orc_alpha(double *out) {
  out[0] = ALPHA[0];
  out[1] = ALPHA[1];
  out[2] = ALPHA[2];
}

/* ------------------------------------------------------------------------- */
/* Multi-resolution WENO, fifth order (Section 3.3; only cited by the paper)  */
/* ------------------------------------------------------------------------- */

/* Left limit at x_{i+1/2} from w_{i-2..i+2} treated as cell averages.  Levels:
 * q1 (1 point, degree 0), q2 (3 points, degree 2), q3 (5 points, degree 4), with
 * linear weights lam[2], lam[1], lam[0] respectively; beta are Jiang-Shu smoothness
 * functionals (beta1 of the 1-point level is the smaller squared one-sided
 * difference); tau = ((|b3 - b1| + |b3 - b2|)/2)^2; wbar_l = lam_l (1 + tau/(b_l + eps)). */
double orc_mrweno5(const orc_cfg *c, double wm2, double wm1, double w0, double w1, double w2) {
  double q1 = w0;
  double q2 = (-wm1 + 5.0 * w0 + 2.0 * w1) / 6.0;
  double q3 = (2.0 * wm2 - 13.0 * wm1 + 47.0 * w0 + 27.0 * w1 - 3.0 * w2) / 60.0;
  double dl = w0 - wm1, dr = w1 - w0;
  double b1 = fmin(dl * dl, dr * dr);
  double t1 = wm1 - 2.0 * w0 + w1, t2 = w1 - wm1;
  double b2 = 13.0 / 12.0 * t1 * t1 + 0.25 * t2 * t2;
  /* b3 depends only on derivatives of the quartic, so it is unchanged when a constant is added
     to the data; it is evaluated on the data relative to the centre value w0, which is the
     same quadratic form without the cancellation between terms of the size of the data's
     square (entropy-variable data carry large offsets, c_v ln T) */
  double am = wm2 - w0, bm = wm1 - w0, cp = w1 - w0, dp = w2 - w0;
  double b3 = (104963.0 * (bm * bm + cp * cp) - 51001.0 * (bm * am + cp * dp)
               + 179098.0 * bm * cp - 38947.0 * (bm * dp + am * cp)
               + 6908.0 * (am * am + dp * dp) + 8209.0 * am * dp) / 5040.0;
  double tt = 0.5 * (fabs(b3 - b1) + fabs(b3 - b2));
  double tau = tt * tt;
  double eps = c->weno_eps;
  double lam0 = c->weno_lin[0], lam1 = c->weno_lin[1], lam2 = c->weno_lin[2];
  double o0 = lam0 * (1.0 + tau / (b3 + eps));
  double o1 = lam1 * (1.0 + tau / (b2 + eps));
  double o2 = lam2 * (1.0 + tau / (b1 + eps));
  double s = o0 + o1 + o2;
  o0 /= s;
  o1 /= s;
  o2 /= s;
  double p3 = (q3 - lam1 * q2 - lam2 * q1) / lam0;
  return o0 * p3 + o1 * q2 + o2 * q1;
}

/* ------------------------------------------------------------------------- */
/* Scaled eigenvectors and rotation (Section 3.3, eq. eigen)                  */
/* ------------------------------------------------------------------------- */

/* 5x5 rotation T of Section 3.3 built from the angles theta and varphi of the metric
   vector n, then restricted to the d active velocity components.  Tr[r*NVMAX+s]. */
static void rotation(int d, const double *n, double *Tr) {
  double n1 = n[0], n2 = d > 1 ? n[1] : 0.0, n3 = d > 2 ? n[2] : 0.0;
  double th = atan2(n2, n1);
  double ph = atan2(n3, sqrt(n1 * n1 + n2 * n2));
  double T5[5][5] = {
      {1, 0, 0, 0, 0},
      {0, cos(ph) * cos(th), cos(ph) * sin(th), sin(ph), 0},
      {0, -sin(th), cos(th), 0, 0},
      {0, -sin(ph) * cos(th), -sin(ph) * sin(th), cos(ph), 0},
      {0, 0, 0, 0, 1}};
  int map[NVMAX];
  int nv = d + 2;
  for (int i = 0; i <= d; ++i) map[i] = i;
  map[d + 1] = 4;
  for (int r = 0; r < nv; ++r)
    for (int s = 0; s < nv; ++s) Tr[r * NVMAX + s] = T5[map[r]][map[s]];
}

/* Scaled right eigenvector matrix R = R~ S of dF_1/dU at the (already rotated) state
 * (rho, u (d comps), p), and its eigenvalues.  Returns 0 if S^2 has a non-positive entry. */
int orc_eigen(const orc_cfg *c, double rho, const double *u, double p, double *Rm, double *lam) {
  int d = c->dim, nv = d + 2;
  double T = orc_T_from_rho_p(c, rho, p);
  double c2 = eos_sound2(c, rho, T);
  double ob = 1.0 - c->b * rho;
  double v2 = 0.0;
  for (int m = 0; m < d; ++m) v2 += u[m] * u[m];
  double E = rho * eos_energy(c, rho, T) + 0.5 * rho * v2;
  double H = (E + p) / rho;
  double Gam = c->R / (c->cv * ob); /* (dp/de)_rho / rho */
  double cs = sqrt(c2);
  double un = u[0];
  double Rt[NVMAX * NVMAX];
  memset(Rt, 0, sizeof(Rt));
  /* column 0: lambda = u_n - c */
  Rt[0 * NVMAX + 0] = 1.0;
  Rt[1 * NVMAX + 0] = un - cs;
  for (int m = 1; m < d; ++m) Rt[(1 + m) * NVMAX + 0] = u[m];
  Rt[(d + 1) * NVMAX + 0] = H - un * cs;
  /* column 1: lambda = u_n (entropy wave) */
  Rt[0 * NVMAX + 1] = 1.0;
  Rt[1 * NVMAX + 1] = un;
  for (int m = 1; m < d; ++m) Rt[(1 + m) * NVMAX + 1] = u[m];
  Rt[(d + 1) * NVMAX + 1] = H - c2 / Gam;
  /* columns 2..d: lambda = u_n (shear waves) */
  for (int m = 1; m < d; ++m) {
    Rt[(1 + m) * NVMAX + (1 + m)] = 1.0;
    Rt[(d + 1) * NVMAX + (1 + m)] = u[m];
  }
  /* column d+1: lambda = u_n + c */
  Rt[0 * NVMAX + (d + 1)] = 1.0;
  Rt[1 * NVMAX + (d + 1)] = un + cs;
  for (int m = 1; m < d; ++m) Rt[(1 + m) * NVMAX + (d + 1)] = u[m];
  Rt[(d + 1) * NVMAX + (d + 1)] = H + un * cs;
  /* S^2: dU/dV = R~ S^2 R~^T */
  double S2[NVMAX];
  double ac = c->R * T - 2.0 * c->a * rho * ob * ob;
  S2[0] = rho * T / (2.0 * c2);
  S2[1] = c->R * c->R * rho * T * T / (c->cv * ac * c2);
  for (int m = 1; m < d; ++m) S2[1 + m] = rho * T;
  S2[d + 1] = rho * T / (2.0 * c2);
  int ok = 1;
  for (int i = 0; i < nv; ++i)
    if (!(S2[i] > 0.0)) ok = 0;
  for (int r = 0; r < nv; ++r)
    for (int s = 0; s < nv; ++s) Rm[r * NVMAX + s] = Rt[r * NVMAX + s] * sqrt(fabs(S2[s]));
  lam[0] = un - cs;
  for (int m = 0; m < d; ++m) lam[1 + m] = un;
  lam[d + 1] = un + cs;
  return ok;
}

/* ------------------------------------------------------------------------- */
/* Grid, padded arrays, boundary conditions                                   */
/* ------------------------------------------------------------------------- */

typedef struct {
  int d;
  int n[3];
  int g[3];  /* ghost width in each direction (0 when the direction is inactive) */
  int P[3];  /* padded extent */
  long N;    /* padded node count */
} pad_t;

static pad_t make_pad(const orc_cfg *c, int g) {
  pad_t p;
  p.d = c->dim;
  for (int k = 0; k < 3; ++k) {
    p.n[k] = k < c->dim ? c->n[k] : 1;
    p.g[k] = k < c->dim ? g : 0;
    p.P[k] = p.n[k] + 2 * p.g[k];
  }
  p.N = (long)p.P[0] * p.P[1] * p.P[2];
  return p;
}

static long pidx(const pad_t *p, int i0, int i1, int i2) {
  return ((long)(i2 + p->g[2]) * p->P[1] + (i1 + p->g[1])) * p->P[0] + (i0 + p->g[0]);
}

static long nodes(const orc_cfg *c) {
  long N = 1;
  for (int k = 0; k < c->dim; ++k) N *= c->n[k];
  return N;
}

static long iidx(const orc_cfg *c, int i0, int i1, int i2) {
  int n0 = c->n[0], n1 = c->dim > 1 ? c->n[1] : 1;
  return ((long)i2 * n1 + i1) * n0 + i0;
}

static double dxi(const orc_cfg *c, int k) { return (c->hi[k] - c->lo[k]) / c->n[k]; }

/* ------------------------------------------------------------------------- */
/* Backward-facing step (Example 5.5; its geometry is a reading, see orc_cfg)  */
/* ------------------------------------------------------------------------- */

static int has_step(const orc_cfg *c) { return c->dim == 2 && c->step[0] > 0 && c->step[1] > 0; }

/* node (i0, i1) lies in the solid block (indices may lie outside the grid) */
static int solid(const orc_cfg *c, int i0, int i1) {
  return has_step(c) && i0 < c->step[0] && i1 < c->step[1];
}

/* Seen along direction k, a solid node within 3 nodes of the step's face normal to k is the
 * mirror image of a fluid node across that face (as a ghost node beyond a wall face of the
 * domain is): returns 1 and the source's index along k in *src, else 0.  Along a line the
 * fluid nodes form a suffix, so the images are the 3 solid nodes next to the first fluid one. */
static int step_image(const orc_cfg *c, int k, int i0, int i1, int *src) {
  if (!solid(c, i0, i1)) return 0;
  if (k == 0 && i0 >= c->step[0] - 3) {
    *src = 2 * c->step[0] - 1 - i0;
    return 1;
  }
  if (k == 1 && i1 >= c->step[1] - 3) {
    *src = 2 * c->step[1] - 1 - i1;
    return 1;
  }
  return 0;
}

/* State at the solid nodes within 3 of a face of the step: the image across that face of its
 * fluid source (normal momentum reversed, J copied); the corner block, within 3 of both
 * faces, takes the image across the vertical face (i0 = step[0]).  These values feed the
 * monitor and keep the solid nodes admissible; the fluxes form the images along each direction
 * themselves (rhs_padded).  Other solid nodes keep their values. */
void orc_step_fill_state(const orc_cfg *c, double *JU, double *J) {
  if (!has_step(c)) return;
  long N = nodes(c);
  for (int k = 1; k >= 0; --k)
    for (int i1 = 0; i1 < c->step[1]; ++i1)
      for (int i0 = 0; i0 < c->step[0]; ++i0) {
        int src;
        if (!step_image(c, k, i0, i1, &src)) continue;
        long q = iidx(c, i0, i1, 0), qs = iidx(c, k == 0 ? src : i0, k == 1 ? src : i1, 0);
        for (int v = 0; v < 4; ++v) JU[v * N + q] = (v == 1 + k ? -JU[v * N + qs] : JU[v * N + qs]);
        J[q] = J[qs];
      }
}

/* a scalar node field (the monitor) at the same solid nodes: the value of the source */
void orc_step_fill_scalar(const orc_cfg *c, double *w) {
  if (!has_step(c)) return;
  for (int k = 1; k >= 0; --k)
    for (int i1 = 0; i1 < c->step[1]; ++i1)
      for (int i0 = 0; i0 < c->step[0]; ++i0) {
        int src;
        if (!step_image(c, k, i0, i1, &src)) continue;
        w[iidx(c, i0, i1, 0)] = w[iidx(c, k == 0 ? src : i0, k == 1 ? src : i1, 0)];
      }
}

/* Mesh at the solid nodes and at the corner, so that the stencils of the fluid nodes (metrics,
 * monitor, Jacobi sweeps) see the image of the mesh across each face.
 *
 * The 6 x 6 block of nodes within 3 of the corner along both directions (the solid corner
 * nodes and the three 3 x 3 fluid blocks left-above, right-above and right-below of the corner)
 * is a lattice mirror-symmetric about both faces: x_1 = face_1 +- a_m on the columns
 * step[0] + m and step[0] - 1 - m, x_2 = face_2 +- b_m on the rows step[1] + m and
 * step[1] - 1 - m (m = 0, 1, 2).  A solid corner node is the image of a fluid node across
 * the vertical face and of another across the horizontal one, and the metric stencils of the
 * fluid nodes near the corner use it in both roles; on such a lattice both images are the same
 * point, so the discrete metric identities and the zero normal flux through both faces hold
 * exactly.  a_m is the mean of the 9 distances to the vertical face of the fluid nodes of the
 * block on the two columns of index m (6 on the right, 3 on the left), b_m likewise for the
 * rows; a lattice is left as it is, up to rounding.
 *
 * A solid node within 3 of one face only holds the image of its source (normal coordinate
 * 2 face - x, the other unchanged); the other solid nodes hold their uniform positions. */
void orc_step_fill_mesh(const orc_cfg *c, double *x) {
  if (!has_step(c)) return;
  long N = nodes(c);
  int s0 = c->step[0], s1 = c->step[1];
  double face[2] = {c->lo[0] + s0 * dxi(c, 0), c->lo[1] + s1 * dxi(c, 1)};
  double a[3], b[3];
  for (int m = 0; m < 3; ++m) {
    double sa = 0.0, sb = 0.0;
    for (int k = -3; k < 3; ++k) sa += x[iidx(c, s0 + m, s1 + k, 0)] - face[0];
    for (int k = 0; k < 3; ++k) sa += face[0] - x[iidx(c, s0 - 1 - m, s1 + k, 0)];
    for (int k = -3; k < 3; ++k) sb += x[N + iidx(c, s0 + k, s1 + m, 0)] - face[1];
    for (int k = 0; k < 3; ++k) sb += face[1] - x[N + iidx(c, s0 + k, s1 - 1 - m, 0)];
    a[m] = sa / 9.0;
    b[m] = sb / 9.0;
  }
  for (int i1 = s1 - 3; i1 < s1 + 3; ++i1)
    for (int i0 = s0 - 3; i0 < s0 + 3; ++i0) {
      long q = iidx(c, i0, i1, 0);
      x[q] = i0 >= s0 ? face[0] + a[i0 - s0] : face[0] - a[s0 - 1 - i0];
      x[N + q] = i1 >= s1 ? face[1] + b[i1 - s1] : face[1] - b[s1 - 1 - i1];
    }
  for (int i1 = 0; i1 < s1; ++i1)
    for (int i0 = 0; i0 < s0; ++i0) {
      if (i0 >= s0 - 3 && i1 >= s1 - 3) continue; /* the corner lattice */
      long q = iidx(c, i0, i1, 0);
      int s, row = step_image(c, 0, i0, i1, &s), col = step_image(c, 1, i0, i1, &s);
      if (row == col) { /* deep inside */
        x[q] = c->lo[0] + (i0 + 0.5) * dxi(c, 0);
        x[N + q] = c->lo[1] + (i1 + 0.5) * dxi(c, 1);
        continue;
      }
      int k = row ? 0 : 1, src;
      step_image(c, k, i0, i1, &src);
      long qs = iidx(c, k == 0 ? src : i0, k == 1 ? src : i1, 0);
      for (int j = 0; j < 2; ++j) x[j * N + q] = j == k ? 2.0 * face[k] - x[j * N + qs] : x[j * N + qs];
    }
}

/* Fill the ghost layers of nf padded scalar fields, direction by direction.
 * kind 0: state field (periodic wrap, outflow: nearest interior node; reflecting wall face:
 *         mirror image, sign reversed when the field is the momentum component `coord` == k;
 *         coord = -1 for fields that are not momentum components).
 * kind 1: mesh coordinate field number `coord` (periodic: shift by one period when
 *         coord == k; outflow and walls: mirror about the boundary face, odd in coord == k).
 * kind 2: mesh velocity component `coord` (periodic: plain wrap; outflow: mirror, odd).
 * kind 3: scalar replicate/wrap, mirror at a wall face (used for the monitor). */
static void fill_ghosts(const orc_cfg *c, const pad_t *p, double *f, int kind, int coord) {
  for (int k = 0; k < c->dim; ++k) {
    int n = p->n[k], g = p->g[k];
    /* loop over all padded positions in directions already filled, interior in later ones */
    int lo[3], hi[3];
    for (int q = 0; q < 3; ++q) {
      if (q < k) { lo[q] = -p->g[q]; hi[q] = p->n[q] + p->g[q]; }
      else { lo[q] = 0; hi[q] = p->n[q]; }
    }
    lo[k] = 0; hi[k] = 1; /* the direction k index is set below */
    for (int i2 = lo[2]; i2 < hi[2]; ++i2)
      for (int i1 = lo[1]; i1 < hi[1]; ++i1)
        for (int i0 = lo[0]; i0 < hi[0]; ++i0) {
          int base[3] = {i0, i1, i2};
          for (int gi = 1; gi <= g; ++gi) {
            for (int side = 0; side < 2; ++side) {
              int ig = side == 0 ? -gi : n - 1 + gi; /* ghost index */
              int is;                               /* source interior index */
              double sgn = 1.0, shift = 0.0;
              if (c->bc[k] == BC_PERIODIC) {
                is = side == 0 ? ig + n : ig - n;
                if (kind == 1 && coord == k) shift = side == 0 ? -(c->hi[k] - c->lo[k]) : (c->hi[k] - c->lo[k]);
              } else {
                int wall = (c->walls >> (2 * k + side)) & 1;
                if ((kind == 0 || kind == 3) && wall) {
                  /* reflecting wall: mirror image, normal momentum reversed */
                  is = side == 0 ? -1 - ig : 2 * n - 1 - ig;
                  if (kind == 0 && coord == k) sgn = -1.0;
                } else if (kind == 0 || kind == 3) {
                  is = side == 0 ? 0 : n - 1;
                } else {
                  is = side == 0 ? -1 - ig : 2 * n - 1 - ig;
                  if (coord == k) {
                    sgn = -1.0;
                    if (kind == 1) shift = 2.0 * (side == 0 ? c->lo[k] : c->hi[k]);
                  }
                }
              }
              int a[3] = {base[0], base[1], base[2]}, s[3] = {base[0], base[1], base[2]};
              a[k] = ig;
              s[k] = is;
              f[pidx(p, a[0], a[1], a[2])] = shift + sgn * f[pidx(p, s[0], s[1], s[2])];
            }
          }
        }
  }
}

/* copy an interior field into the interior of a padded field */
static void to_pad(const orc_cfg *c, const pad_t *p, const double *src, double *dst) {
  for (int i2 = 0; i2 < p->n[2]; ++i2)
    for (int i1 = 0; i1 < p->n[1]; ++i1)
      for (int i0 = 0; i0 < p->n[0]; ++i0) dst[pidx(p, i0, i1, i2)] = src[iidx(c, i0, i1, i2)];
}

/* ------------------------------------------------------------------------- */
/* Discrete metrics (Section 3.2, eq. SCLCoeff, eq. VCLCoeff)                 */
/* ------------------------------------------------------------------------- */

/* delta_k[a]_i = 1/2 sum_m alpha_m (a_{i+m e_k} - a_{i-m e_k}) on a padded field */
static double delta_op(const pad_t *p, const double *a, int k, int i0, int i1, int i2) {
  double s = 0.0;
  for (int m = 1; m <= 3; ++m) {
    int ip[3] = {i0, i1, i2}, im[3] = {i0, i1, i2};
    ip[k] += m;
    im[k] -= m;
    s += ALPHA[m - 1] * (a[pidx(p, ip[0], ip[1], ip[2])] - a[pidx(p, im[0], im[1], im[2])]);
  }
  return 0.5 * s;
}

/* Metrics J xi_k/x_j at every node of the padded grid pm (ghost width GS), from the
 * mesh x padded with width GM.  met[(k*d + j)*pm.N + idx].  In 3D the conservative
 * nested form (delta_{k+2}[delta_{k+1}[x_{j+1}] x_{j+2}] - delta_{k+1}[delta_{k+2}[x_{j+1}]
 * x_{j+2}])/(dxi_{k+1} dxi_{k+2}) with cyclic indices. */
static void metrics_padded(const orc_cfg *c, const pad_t *px, double *const *xp, const pad_t *pm, double *met) {
  int d = c->dim;
  double dx[3];
  for (int k = 0; k < d; ++k) dx[k] = dxi(c, k);
  if (d == 3) {
    /* products delta_q[x_r] * x_s, computed on the mesh padding less 3 layers */
    double *tmp = malloc(sizeof(double) * px->N);
    for (int k = 0; k < 3; ++k) {
      int k1 = (k + 1) % 3, k2 = (k + 2) % 3;
      for (int j = 0; j < 3; ++j) {
        int j1 = (j + 1) % 3, j2 = (j + 2) % 3;
        double *outp = met + (long)(k * 3 + j) * pm->N;
        for (long q = 0; q < pm->N; ++q) outp[q] = 0.0;
        for (int term = 0; term < 2; ++term) {
          int inner = term == 0 ? k1 : k2; /* delta_inner[x_j1] * x_j2 then delta_outer */
          int outer = term == 0 ? k2 : k1;
          double sg = term == 0 ? 1.0 : -1.0;
          /* the product is needed 3 + GS layers out along `outer` and GS layers out
             along the other two directions; delta_inner reads 3 more along `inner` */
          for (long q = 0; q < px->N; ++q) tmp[q] = 0.0;
#pragma omp parallel for schedule(static)
          for (int i2 = -GM; i2 < px->n[2] + GM; ++i2)
            for (int i1 = -GM; i1 < px->n[1] + GM; ++i1)
              for (int i0 = -GM; i0 < px->n[0] + GM; ++i0) {
                int ii[3] = {i0, i1, i2};
                if (ii[inner] < -GS || ii[inner] >= px->n[inner] + GS) continue;
                long q = pidx(px, i0, i1, i2);
                tmp[q] = delta_op(px, xp[j1], inner, i0, i1, i2) * xp[j2][q];
              }
#pragma omp parallel for schedule(static)
          for (int i2 = -GS; i2 < pm->n[2] + GS; ++i2)
            for (int i1 = -GS; i1 < pm->n[1] + GS; ++i1)
              for (int i0 = -GS; i0 < pm->n[0] + GS; ++i0)
                outp[pidx(pm, i0, i1, i2)] += sg * delta_op(px, tmp, outer, i0, i1, i2) / (dx[k1] * dx[k2]);
        }
      }
    }
    free(tmp);
    return;
  }
#pragma omp parallel for collapse(2) schedule(static)
  for (int i2 = -pm->g[2]; i2 < pm->n[2] + pm->g[2]; ++i2)
    for (int i1 = -pm->g[1]; i1 < pm->n[1] + pm->g[1]; ++i1)
      for (int i0 = -pm->g[0]; i0 < pm->n[0] + pm->g[0]; ++i0) {
        long q = pidx(pm, i0, i1, i2);
        if (d == 1) {
          met[q] = 1.0; /* J xi_x = 1 in one dimension */
        } else {
          double d1x1 = delta_op(px, xp[0], 0, i0, i1, i2), d1x2 = delta_op(px, xp[1], 0, i0, i1, i2);
          double d2x1 = delta_op(px, xp[0], 1, i0, i1, i2), d2x2 = delta_op(px, xp[1], 1, i0, i1, i2);
          met[0 * pm->N + q] = d2x2 / dx[1];  /* J xi_1/x_1 =  x_2,xi2 */
          met[1 * pm->N + q] = -d2x1 / dx[1]; /* J xi_1/x_2 = -x_1,xi2 */
          met[2 * pm->N + q] = -d1x2 / dx[0]; /* J xi_2/x_1 = -x_2,xi1 */
          met[3 * pm->N + q] = d1x1 / dx[0];  /* J xi_2/x_2 =  x_1,xi1 */
        }
      }
}

/* build the GM-padded mesh (and optionally velocity) from interior arrays */
static double **pad_mesh(const orc_cfg *c, const pad_t *px, const double *x, int kind) {
  int d = c->dim;
  long N = nodes(c);
  double **xp = malloc(sizeof(double *) * d);
  for (int j = 0; j < d; ++j) {
    xp[j] = calloc(px->N, sizeof(double));
    to_pad(c, px, x + j * N, xp[j]);
    fill_ghosts(c, px, xp[j], kind, j);
  }
  return xp;
}

static void free_fields(double **f, int nf) {
  for (int j = 0; j < nf; ++j) free(f[j]);
  free(f);
}

/* interior metrics: met[(k*d+j)*N], xit[k*N] (xit may be NULL; xdot NULL means 0) */
void orc_metrics(const orc_cfg *c, const double *x, const double *xdot, double *met, double *xit) {
  int d = c->dim;
  long N = nodes(c);
  pad_t px = make_pad(c, GM), pm = make_pad(c, GS);
  double **xp = pad_mesh(c, &px, x, 1);
  double *mp = malloc(sizeof(double) * d * d * pm.N);
  metrics_padded(c, &px, xp, &pm, mp);
  for (int i2 = 0; i2 < pm.n[2]; ++i2)
    for (int i1 = 0; i1 < pm.n[1]; ++i1)
      for (int i0 = 0; i0 < pm.n[0]; ++i0) {
        long qi = iidx(c, i0, i1, i2), qp = pidx(&pm, i0, i1, i2);
        for (int kj = 0; kj < d * d; ++kj) met[kj * N + qi] = mp[kj * pm.N + qp];
        if (xit) {
          for (int k = 0; k < d; ++k) {
            double s = 0.0;
            if (xdot)
              for (int j = 0; j < d; ++j) s -= xdot[j * N + qi] * mp[(k * d + j) * pm.N + qp];
            xit[k * N + qi] = s;
          }
        }
      }
  free(mp);
  free_fields(xp, d);
}

/* discrete Jacobian J = det(dx/dxi) from the same delta operators: 1D delta_1[x]/dxi;
   2D (delta_1[x_1] delta_2[x_2] - delta_2[x_1] delta_1[x_2])/(dxi_1 dxi_2);
   3D sum_j (delta_1[x_j]/dxi_1) (J xi_1/x_j). */
void orc_jacobian(const orc_cfg *c, const double *x, double *J) {
  int d = c->dim;
  pad_t px = make_pad(c, GM), pm = make_pad(c, GS);
  double **xp = pad_mesh(c, &px, x, 1);
  double *mp = d == 3 ? malloc(sizeof(double) * 9 * pm.N) : NULL;
  if (d == 3) metrics_padded(c, &px, xp, &pm, mp);
  for (int i2 = 0; i2 < pm.n[2]; ++i2)
    for (int i1 = 0; i1 < pm.n[1]; ++i1)
      for (int i0 = 0; i0 < pm.n[0]; ++i0) {
        long qi = iidx(c, i0, i1, i2);
        double v;
        if (d == 1) {
          v = delta_op(&px, xp[0], 0, i0, i1, i2) / dxi(c, 0);
        } else if (d == 2) {
          v = (delta_op(&px, xp[0], 0, i0, i1, i2) * delta_op(&px, xp[1], 1, i0, i1, i2)
               - delta_op(&px, xp[0], 1, i0, i1, i2) * delta_op(&px, xp[1], 0, i0, i1, i2)) / (dxi(c, 0) * dxi(c, 1));
        } else {
          v = 0.0;
          for (int j = 0; j < 3; ++j) v += delta_op(&px, xp[j], 0, i0, i1, i2) / dxi(c, 0) * mp[j * pm.N + pidx(&pm, i0, i1, i2)];
        }
        J[qi] = v;
      }
  free(mp);
  free_fields(xp, d);
}

/* uniform mesh x = xi at the cell-centred nodes */
void orc_uniform_mesh(const orc_cfg *c, double *x) {
  int d = c->dim;
  long N = nodes(c);
  int n1 = d > 1 ? c->n[1] : 1, n2 = d > 2 ? c->n[2] : 1;
  for (int i2 = 0; i2 < n2; ++i2)
    for (int i1 = 0; i1 < n1; ++i1)
      for (int i0 = 0; i0 < c->n[0]; ++i0) {
        int ii[3] = {i0, i1, i2};
        for (int j = 0; j < d; ++j) x[j * N + iidx(c, i0, i1, i2)] = c->lo[j] + (ii[j] + 0.5) * dxi(c, j);
      }
  orc_step_fill_mesh(c, x);
}

/* ------------------------------------------------------------------------- */
/* Semi-discrete right-hand side (eq. semi_U, eq. semi_J, eq. HOstable)       */
/* ------------------------------------------------------------------------- */

/* One interface i+1/2 in direction k.  st[s] (s = 0..5 <-> nodes i-2..i+3) hold the
 * conserved state, mx[s][j] = J xi_k/x_j and mt[s] = J xi_k/t of those nodes.
 * Outputs the entropy-stable flux Fes[nv] and the GCL flux of J xi_k/t.  Returns the
 * interface entropy production sum_m [W_m] Y_m [W_m]^WENO * Lambda / 2 in *prod.
 * diag (may be NULL; 4 NVMAX doubles) receives, per component m, the sign-matrix entry Y_m,
 * the reconstructed jump [W_m]^WENO, the plain jump [W_m] before the zero test and the
 * rounding scale of W_m used by that test (for tests of the dissipation's switch). */
static void interface_flux(const orc_cfg *c, double st[6][NVMAX], double mx[6][3], const double *mt,
                           double *Fes, double *gclt, double *prod, double *diag) {
  int d = c->dim, nv = d + 2;
  /* eq. ECFlux_curv_2p and eq. GCL_flux with w = 3; node offset o <-> index i + o - 2 */
  double Fec[NVMAX] = {0}, gt = 0.0;
  for (int m = 1; m <= 3; ++m)
    for (int s = 0; s <= m - 1; ++s) {
      int l = 2 - s, r = 2 - s + m; /* nodes i - s and i - s + m */
      double Fh[NVMAX];
      ec_pair_curv(c, st[l], st[r], mt[l], mt[r], mx[l], mx[r], Fh);
      for (int q = 0; q < nv; ++q) Fec[q] += ALPHA[m - 1] * Fh[q];
      gt += ALPHA[m - 1] * 0.5 * (mt[l] + mt[r]);
    }
  *gclt = gt;
  for (int q = 0; q < nv; ++q) Fes[q] = Fec[q];
  *prod = 0.0;
  if (diag)
    for (int q = 0; q < 4 * NVMAX; ++q) diag[q] = 0.0;
  if (!c->dissipation) return;

  /* averaged state at i+1/2: rho = L(rho), v = {v}, p = L(rho)/L(rho/p) */
  double z[6][NVMAX], pr[6];
  for (int s = 0; s < 6; ++s) {
    cons_to_z(c, st[s], z[s]);
    pr[s] = eos_pressure(c, z[s][0], z[s][d + 1]);
  }
  double rb = orc_logmean(z[2][0], z[3][0]);
  double pb = rb / orc_logmean(z[2][0] / pr[2], z[3][0] / pr[3]);
  double vb[3];
  for (int m = 0; m < d; ++m) vb[m] = 0.5 * (z[2][1 + m] + z[3][1 + m]);
  /* interface metrics: arithmetic mean of the two nodes */
  double mm[3], L = 0.0, mtb = 0.5 * (mt[2] + mt[3]);
  for (int j = 0; j < d; ++j) {
    mm[j] = 0.5 * (mx[2][j] + mx[3][j]);
    L += mm[j] * mm[j];
  }
  L = sqrt(L);
  double nrm[3] = {0.0, 0.0, 0.0};
  for (int j = 0; j < d; ++j) nrm[j] = mm[j] / L;
  double Tm[NVMAX * NVMAX];
  rotation(d, nrm, Tm);
  /* rotated average state T U: rotate the velocity */
  double ub[3];
  for (int r = 0; r < d; ++r) {
    double s = 0.0;
    for (int m = 0; m < d; ++m) s += Tm[(1 + r) * NVMAX + (1 + m)] * vb[m];
    ub[r] = s;
  }
  double Rm[NVMAX * NVMAX], lam[NVMAX];
  if (!orc_eigen(c, rb, ub, pb, Rm, lam)) raise_flag(F_MEANCONSTRAINT);
  double Lam = 0.0;
  for (int q = 0; q < nv; ++q) {
    double v = fabs(mtb + L * lam[q]);
    if (v > Lam) Lam = v;
  }
  /* scaled entropy variables W_s = R^T T V_s on the stencil; Wmag_s = |R|^T |T V_s| bounds
     the magnitude of the terms summed into W_s (used for the zero test of Y below) */
  double W[6][NVMAX], Wmag[6][NVMAX];
  for (int s = 0; s < 6; ++s) {
    double V[NVMAX], TV[NVMAX];
    orc_entropy_vars(c, st[s], V);
    for (int r = 0; r < nv; ++r) {
      double a = 0.0;
      for (int q = 0; q < nv; ++q) a += Tm[r * NVMAX + q] * V[q];
      TV[r] = a;
    }
    for (int r = 0; r < nv; ++r) {
      double a = 0.0, m = 0.0;
      for (int q = 0; q < nv; ++q) {
        a += Rm[q * NVMAX + r] * TV[q];
        m += fabs(Rm[q * NVMAX + r]) * fabs(TV[q]);
      }
      W[s][r] = a;
      Wmag[s][r] = m;
    }
  }
  /* jumps: plain [W] and reconstructed [W]^WENO = W+ - W-; sign matrix Y.  A plain jump
     below the rounding level of the vector W (2^-40 of the magnitude of all the terms that form
     the W components at the two nodes) is taken as zero, so Y = 0 there: Y only gates
     dissipation, so the flux stays entropy stable.  (A component's own terms can all be
     rounding residue of exact zeros, e.g. a tangential velocity that vanishes by symmetry; its
     plain jump is then noise whose sign must not decide Y.) */
  double wscale = 0.0;
  for (int r = 0; r < nv; ++r) wscale += Wmag[2][r] + Wmag[3][r];
  double YdW[NVMAX];
  for (int r = 0; r < nv; ++r) {
    double Wm = orc_mrweno5(c, W[0][r], W[1][r], W[2][r], W[3][r], W[4][r]);
    double Wp = orc_mrweno5(c, W[5][r], W[4][r], W[3][r], W[2][r], W[1][r]);
    double jw = Wp - Wm;
    double j0 = W[3][r] - W[2][r];
    if (diag) {
      diag[NVMAX + r] = jw;
      diag[2 * NVMAX + r] = j0;
      diag[3 * NVMAX + r] = wscale;
    }
    if (fabs(j0) <= ldexp(wscale, -40)) j0 = 0.0;
    int same = (jw > 0.0 && j0 > 0.0) || (jw < 0.0 && j0 < 0.0);
    YdW[r] = same ? jw : 0.0;
    if (diag) diag[r] = same ? 1.0 : 0.0;
    *prod += 0.5 * Lam * j0 * YdW[r];
  }
  /* F_es = F_ec - 1/2 Lambda T^{-1} R Y [W]^WENO, with T^{-1} = T^T */
  double RY[NVMAX];
  for (int r = 0; r < nv; ++r) {
    double a = 0.0;
    for (int q = 0; q < nv; ++q) a += Rm[r * NVMAX + q] * YdW[q];
    RY[r] = a;
  }
  for (int r = 0; r < nv; ++r) {
    double a = 0.0;
    for (int q = 0; q < nv; ++q) a += Tm[q * NVMAX + r] * RY[q];
    Fes[r] -= 0.5 * Lam * a;
  }
}

/* Right-hand side from padded node states Up (nv fields, width GS) and padded
 * metrics metp (d*d fields) and xitp (d fields).  dJU[nv*N], dJ[N].  If prod != NULL
 * it receives, per node, the entropy production of the two faces' share (sum over
 * the domain gives the total dissipation). */
static void rhs_padded(const orc_cfg *c, const pad_t *pm, double *const *Up, const double *metp,
                       const double *xitp, double *dJU, double *dJ, double *prodsum, double *rec) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  for (long q = 0; q < N * nv; ++q) dJU[q] = 0.0;
  for (long q = 0; q < N; ++q) dJ[q] = 0.0;
  double psum = 0.0;
  const int NR = 5 * nv + 1; /* fields of one interface record (see orc_rhs_record) */
  long roff = 0;             /* start of direction k's records */
  for (int k = 0; k < d; ++k) {
    double dk = dxi(c, k);
    int e[3] = {pm->n[0], pm->n[1], pm->n[2]};
    e[k] += 1;
    long nif = (long)e[0] * e[1] * e[2];
    double cellvol = 1.0;
    for (int q = 0; q < d; ++q) cellvol *= dxi(c, q);
    /* lines of interfaces along k, i+1/2 for i = -1 .. n_k - 1; each line writes only its own
       nodes, so with OpenMP (the throughput build) the lines run in parallel */
    const int ka = (k + 1) % 3, kb = (k + 2) % 3;
    const int na = pm->n[ka], nb = pm->n[kb];
#pragma omp parallel for collapse(2) reduction(+ : psum) schedule(static)
    for (int ib = 0; ib < nb; ++ib)
      for (int ia = 0; ia < na; ++ia)
        for (int ik = -1; ik < pm->n[k]; ++ik) {
          int il[3];
          il[k] = ik;
          il[ka] = ia;
          il[kb] = ib;
          const int i0 = il[0], i1 = il[1], i2 = il[2];
          /* with a step, only the faces with a fluid node on their right (the first fluid node
             of a line and beyond) carry a flux */
          if (has_step(c) && solid(c, i0 + (k == 0), i1 + (k == 1))) continue;
          double st[6][NVMAX], mx[6][3], mt[6];
          for (int s = 0; s < 6; ++s) {
            int ii[3] = {i0, i1, i2};
            ii[k] += s - 2;
            /* a solid node next to a face of the step: the mirror image of its fluid source
               across that face (normal momentum, J xi_k/x_j for j != k and J xi_k/t reversed) */
            int src, img = step_image(c, k, ii[0], ii[1], &src);
            if (img) ii[k] = src;
            long qp = pidx(pm, ii[0], ii[1], ii[2]);
            for (int v = 0; v < nv; ++v) st[s][v] = (img && v == 1 + k) ? -Up[v][qp] : Up[v][qp];
            for (int j = 0; j < d; ++j)
              mx[s][j] = (img && j != k) ? -metp[(k * d + j) * pm->N + qp] : metp[(k * d + j) * pm->N + qp];
            mt[s] = img ? -xitp[k * pm->N + qp] : xitp[k * pm->N + qp];
          }
          double Fes[NVMAX], gt, prod, dg[4 * NVMAX];
          interface_flux(c, st, mx, mt, Fes, &gt, &prod, rec ? dg : NULL);
          int ii[3] = {i0, i1, i2};
          if (rec) {
            int a[3] = {i0, i1, i2};
            a[k] += 1;
            long ti = ((long)a[2] * e[1] + a[1]) * e[0] + a[0];
            double *r = rec + roff;
            for (int v = 0; v < nv; ++v) {
              r[(long)v * nif + ti] = Fes[v];
              for (int q = 0; q < 4; ++q) r[(long)(nv + 1 + q * nv + v) * nif + ti] = dg[q * NVMAX + v];
            }
            r[(long)nv * nif + ti] = gt;
          }
          /* the interface contributes -F/dxi to node i and +F/dxi to node i+1 */
          if (ii[k] >= 0) {
            long qi = iidx(c, ii[0], ii[1], ii[2]);
            for (int v = 0; v < nv; ++v) dJU[v * N + qi] -= Fes[v] / dk;
            dJ[qi] -= gt / dk;
          }
          if (ii[k] + 1 < pm->n[k]) {
            int jj[3] = {ii[0], ii[1], ii[2]};
            jj[k] += 1;
            long qi = iidx(c, jj[0], jj[1], jj[2]);
            for (int v = 0; v < nv; ++v) dJU[v * N + qi] += Fes[v] / dk;
            dJ[qi] += gt / dk;
          }
          /* count each interior-domain face once: the i+1/2 faces for i = 0..n-1 */
          if (ii[k] >= 0) psum += prod * cellvol / dk;
        }
    roff += (long)NR * nif;
  }
  /* the solid nodes do not evolve */
  if (has_step(c))
    for (int i1 = 0; i1 < c->step[1]; ++i1)
      for (int i0 = 0; i0 < c->step[0]; ++i0) {
        long qi = iidx(c, i0, i1, 0);
        for (int v = 0; v < nv; ++v) dJU[v * N + qi] = 0.0;
        dJ[qi] = 0.0;
      }
  if (prodsum) *prodsum = psum;
}

/* padded node states from JU, J */
static double **pad_state(const orc_cfg *c, const pad_t *pm, const double *JU, const double *J) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  double **Up = malloc(sizeof(double *) * nv);
  for (int v = 0; v < nv; ++v) {
    Up[v] = calloc(pm->N, sizeof(double));
    for (int i2 = 0; i2 < pm->n[2]; ++i2)
      for (int i1 = 0; i1 < pm->n[1]; ++i1)
        for (int i0 = 0; i0 < pm->n[0]; ++i0) {
          long qi = iidx(c, i0, i1, i2);
          Up[v][pidx(pm, i0, i1, i2)] = JU[v * N + qi] / J[qi];
        }
    fill_ghosts(c, pm, Up[v], 0, v >= 1 && v <= d ? v - 1 : -1);
  }
  if (c->inflow) {
    /* the lo face of direction 0 holds the fixed inflow state in all its ghost layers */
    double pr[NVMAX], Uin[NVMAX];
    for (int v = 0; v < nv; ++v) pr[v] = c->inflow_prim[v];
    orc_prim_to_cons(c, pr, Uin);
    for (int i2 = -pm->g[2]; i2 < pm->n[2] + pm->g[2]; ++i2)
      for (int i1 = -pm->g[1]; i1 < pm->n[1] + pm->g[1]; ++i1)
        for (int i0 = -pm->g[0]; i0 < 0; ++i0)
          for (int v = 0; v < nv; ++v) Up[v][pidx(pm, i0, i1, i2)] = Uin[v];
  }
  return Up;
}

/* Metrics supplied at interior nodes only: extend them to the ghost layers by the
 * symmetry of the boundary condition (periodic: wrap; outflow mirror about the face
 * normal to direction q: J xi_k/x_j changes sign iff exactly one of k, j equals q,
 * J xi_k/t changes sign iff k = q). */
static void pad_metrics(const orc_cfg *c, const pad_t *pm, const double *met, const double *xit,
                        double *metp, double *xitp) {
  int d = c->dim;
  long N = nodes(c);
  for (int f = 0; f < d * d + d; ++f) {
    double *dst = f < d * d ? metp + (long)f * pm->N : xitp + (long)(f - d * d) * pm->N;
    const double *src = f < d * d ? met + (long)f * N : xit + (long)(f - d * d) * N;
    to_pad(c, pm, src, dst);
    /* ghost fill with a per-direction sign */
    for (int q = 0; q < d; ++q) {
      double sg;
      if (f < d * d) {
        int k = f / d, j = f % d;
        sg = ((k == q) != (j == q)) ? -1.0 : 1.0;
      } else {
        int k = f - d * d;
        sg = (k == q) ? -1.0 : 1.0;
      }
      int n = pm->n[q], g = pm->g[q];
      int lo[3], hi[3];
      for (int r = 0; r < 3; ++r) {
        if (r < q) { lo[r] = -pm->g[r]; hi[r] = pm->n[r] + pm->g[r]; }
        else { lo[r] = 0; hi[r] = pm->n[r]; }
      }
      lo[q] = 0; hi[q] = 1;
      for (int i2 = lo[2]; i2 < hi[2]; ++i2)
        for (int i1 = lo[1]; i1 < hi[1]; ++i1)
          for (int i0 = lo[0]; i0 < hi[0]; ++i0)
            for (int gi = 1; gi <= g; ++gi)
              for (int side = 0; side < 2; ++side) {
                int ig = side == 0 ? -gi : n - 1 + gi, is;
                double s = 1.0;
                if (c->bc[q] == BC_PERIODIC) is = side == 0 ? ig + n : ig - n;
                else { is = side == 0 ? -1 - ig : 2 * n - 1 - ig; s = sg; }
                int a[3] = {i0, i1, i2}, b[3] = {i0, i1, i2};
                a[q] = ig;
                b[q] = is;
                dst[pidx(pm, a[0], a[1], a[2])] = s * dst[pidx(pm, b[0], b[1], b[2])];
              }
    }
  }
}

/* RHS with metrics given at the interior nodes (xit may be NULL: static mesh).
   If prod is not NULL it receives the total entropy production (Section 3.3). */
void orc_rhs(const orc_cfg *c, const double *JU, const double *J, const double *met, const double *xit,
             double *dJU, double *dJ, double *prod) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  pad_t pm = make_pad(c, GS);
  double **Up = pad_state(c, &pm, JU, J);
  double *metp = calloc((long)d * d * pm.N, sizeof(double));
  double *xitp = calloc((long)d * pm.N, sizeof(double));
  double *xz = NULL;
  if (!xit) xz = calloc((long)d * N, sizeof(double));
  pad_metrics(c, &pm, met, xit ? xit : xz, metp, xitp);
  rhs_padded(c, &pm, Up, metp, xitp, dJU, dJ, prod, NULL);
  free(xz);
  free(metp);
  free(xitp);
  free_fields(Up, nv);
}

/* The interface records behind orc_rhs, for tests of single interfaces: per direction k, in
 * order, (5 nv + 1) fields over the interfaces of k (e_k = n_k + 1 along k, index
 * (a2 e1 + a1) e0 + a0 with a_k - 1 the left node): the entropy-stable flux (nv), the GCL flux
 * of J xi_k/t (1), then per component Y_m (nv), [W_m]^WENO (nv), the plain jump [W_m] before
 * its zero test (nv) and that test's rounding scale (nv).  dJU, dJ as orc_rhs. */
void orc_rhs_record(const orc_cfg *c, const double *JU, const double *J, const double *met, const double *xit,
                    double *dJU, double *dJ, double *rec) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  pad_t pm = make_pad(c, GS);
  double **Up = pad_state(c, &pm, JU, J);
  double *metp = calloc((long)d * d * pm.N, sizeof(double));
  double *xitp = calloc((long)d * pm.N, sizeof(double));
  double *xz = NULL;
  if (!xit) xz = calloc((long)d * N, sizeof(double));
  pad_metrics(c, &pm, met, xit ? xit : xz, metp, xitp);
  rhs_padded(c, &pm, Up, metp, xitp, dJU, dJ, NULL, rec);
  free(xz);
  free(metp);
  free(xitp);
  free_fields(Up, nv);
}

/* One interface from explicit stencil data (tests): st[6 * nv] conserved states of nodes
 * i-2..i+3, mx[6 * d] their J xi_k/x_j, mt[6] their J xi_k/t.  Outputs as interface_flux;
 * diag (may be NULL) receives 4 nv values: Y, [W]^WENO, plain [W], rounding scale. */
void orc_interface_flux(const orc_cfg *c, const double *st, const double *mx, const double *mt, double *Fes,
                        double *gclt, double *prod, double *diag) {
  int d = c->dim, nv = d + 2;
  double S[6][NVMAX], M[6][3], dg[4 * NVMAX];
  for (int s = 0; s < 6; ++s) {
    for (int v = 0; v < nv; ++v) S[s][v] = st[s * nv + v];
    for (int j = 0; j < 3; ++j) M[s][j] = j < d ? mx[s * d + j] : 0.0;
  }
  interface_flux(c, S, M, mt, Fes, gclt, prod, dg);
  if (diag)
    for (int q = 0; q < 4; ++q)
      for (int v = 0; v < nv; ++v) diag[q * nv + v] = dg[q * NVMAX + v];
}

/* RHS on the stage mesh xs (metrics from the GM-padded mesh, including ghosts) */
static void rhs_on_mesh(const orc_cfg *c, const double *JU, const double *J, const double *xs,
                        const double *xdot, double *dJU, double *dJ) {
  int d = c->dim, nv = d + 2;
  pad_t px = make_pad(c, GM), pm = make_pad(c, GS);
  double **xp = pad_mesh(c, &px, xs, 1);
  double **vp = xdot ? pad_mesh(c, &px, xdot, 2) : NULL;
  double *metp = malloc(sizeof(double) * d * d * pm.N);
  double *xitp = calloc((long)d * pm.N, sizeof(double));
  metrics_padded(c, &px, xp, &pm, metp);
  if (vp) {
    for (int i2 = -pm.g[2]; i2 < pm.n[2] + pm.g[2]; ++i2)
      for (int i1 = -pm.g[1]; i1 < pm.n[1] + pm.g[1]; ++i1)
        for (int i0 = -pm.g[0]; i0 < pm.n[0] + pm.g[0]; ++i0) {
          long qm = pidx(&pm, i0, i1, i2), qx = pidx(&px, i0, i1, i2);
          for (int k = 0; k < d; ++k) {
            double s = 0.0;
            for (int j = 0; j < d; ++j) s -= vp[j][qx] * metp[(k * d + j) * pm.N + qm];
            xitp[k * pm.N + qm] = s;
          }
        }
  }
  double **Up = pad_state(c, &pm, JU, J);
  rhs_padded(c, &pm, Up, metp, xitp, dJU, dJ, NULL, NULL);
  free_fields(Up, nv);
  free(metp);
  free(xitp);
  free_fields(xp, d);
  if (vp) free_fields(vp, d);
}

/* ------------------------------------------------------------------------- */
/* Third-order SSP Runge-Kutta stage (Shu-Osher form; Section 5 cites it)     */
/* ------------------------------------------------------------------------- */

/* Stage s in {0,1,2}: the RHS is evaluated for (JUs, Js) on the mesh x^n + c_s dt xdot,
 * c = (0, 1, 1/2), then combined with the step's base (JU0, J0):
 *   s=0: out = base + dt L;  s=1: out = 3/4 base + 1/4 (in + dt L);
 *   s=2: out = 1/3 base + 2/3 (in + dt L).
 * xdot may be NULL (static mesh).  out may alias the base but not the input. */
void orc_rk_stage(const orc_cfg *c, int s, double dt, const double *JU0, const double *J0,
                  const double *JUs, const double *Js, const double *xn, const double *xdot,
                  double *JUout, double *Jout) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  static const double cst[3] = {0.0, 1.0, 0.5};
  double *xs = malloc(sizeof(double) * d * N);
  for (long q = 0; q < d * N; ++q) xs[q] = xn[q] + (xdot ? cst[s] * dt * xdot[q] : 0.0);
  double *LU = malloc(sizeof(double) * nv * N), *LJ = malloc(sizeof(double) * N);
  rhs_on_mesh(c, JUs, Js, xs, xdot, LU, LJ);
  double a0, a1;
  if (s == 0) { a0 = 0.0; a1 = 1.0; }
  else if (s == 1) { a0 = 0.75; a1 = 0.25; }
  else { a0 = 1.0 / 3.0; a1 = 2.0 / 3.0; }
  for (long q = 0; q < nv * N; ++q) {
    double y = JUs[q] + dt * LU[q];
    JUout[q] = s == 0 ? y : a0 * JU0[q] + a1 * y;
  }
  for (long q = 0; q < N; ++q) {
    double y = Js[q] + dt * LJ[q];
    Jout[q] = s == 0 ? y : a0 * J0[q] + a1 * y;
  }
  if (has_step(c)) {
    /* solid nodes keep the step's base values; those next to the step then take their images */
    for (int i1 = 0; i1 < c->step[1]; ++i1)
      for (int i0 = 0; i0 < c->step[0]; ++i0) {
        long q = iidx(c, i0, i1, 0);
        for (int v = 0; v < nv; ++v) JUout[v * N + q] = JU0[v * N + q];
        Jout[q] = J0[q];
      }
    orc_step_fill_state(c, JUout, Jout);
  }
  free(xs);
  free(LU);
  free(LJ);
}

/* ------------------------------------------------------------------------- */
/* Time step (eq. cfl)                                                        */
/* ------------------------------------------------------------------------- */

/* dt = CFL / max_i sum_k rho_{i,k}/dxi_k, rho_{i,k} = L_k (|v . n_k| + c)/J */
double orc_cfl_dt(const orc_cfg *c, const double *JU, const double *J, const double *x) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  double *met = malloc(sizeof(double) * d * d * N);
  orc_metrics(c, x, NULL, met, NULL);
  double mx = 0.0;
  for (long q = 0; q < N; ++q) {
    if (has_step(c) && solid(c, (int)(q % c->n[0]), (int)(q / c->n[0]))) continue; /* fluid nodes only */
    double U[NVMAX], z[NVMAX];
    for (int v = 0; v < nv; ++v) U[v] = JU[v * N + q] / J[q];
    cons_to_z(c, U, z);
    double cs = sqrt(eos_sound2(c, z[0], z[d + 1]));
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      double L = 0.0, vn = 0.0;
      for (int j = 0; j < d; ++j) {
        double m = met[(k * d + j) * N + q];
        L += m * m;
        vn += m * z[1 + j];
      }
      L = sqrt(L);
      s += (fabs(vn) + L * cs) / J[q] / dxi(c, k);
    }
    if (s > mx) mx = s;
  }
  free(met);
  return c->cfl / mx;
}

/* ------------------------------------------------------------------------- */
/* Adaptive moving mesh (Section 4)                                           */
/* ------------------------------------------------------------------------- */

/* Monitor (eq. van der Waalsmonitor; the smooth tests use eq. van der Waalssinmonitor).
 * Gradients and second derivatives in xi by second-order central differences on the
 * ghost-extended node values; each normalised term is 0 where its maximum is 0. */
void orc_monitor(const orc_cfg *c, const double *JU, const double *J, double *omega) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  pad_t p1 = make_pad(c, 1);
  double *rho = calloc(p1.N, sizeof(double)), *G = calloc(p1.N, sizeof(double));
  double *rhoi = malloc(sizeof(double) * N), *Gi = malloc(sizeof(double) * N);
  for (long q = 0; q < N; ++q) {
    double U[NVMAX], z[NVMAX];
    for (int v = 0; v < nv; ++v) U[v] = JU[v * N + q] / J[q];
    cons_to_z(c, U, z);
    rhoi[q] = z[0];
    Gi[q] = eos_G(c, z[0], z[d + 1]);
  }
  to_pad(c, &p1, rhoi, rho);
  to_pad(c, &p1, Gi, G);
  fill_ghosts(c, &p1, rho, 0, -1);
  fill_ghosts(c, &p1, G, 0, -1);
  int nterm = c->monitor_kind == MON_VDW ? c->kappa + 1 : 2;
  double *term = calloc((long)nterm * N, sizeof(double));
  double mxv[3] = {0, 0, 0};
#pragma omp parallel for collapse(2) reduction(max : mxv[:3]) schedule(static)
  for (int i2 = 0; i2 < p1.n[2]; ++i2)
    for (int i1 = 0; i1 < p1.n[1]; ++i1)
      for (int i0 = 0; i0 < p1.n[0]; ++i0) {
        long qi = iidx(c, i0, i1, i2);
        for (int t = 0; t < nterm; ++t) {
          const double *f;
          int second;
          if (c->monitor_kind == MON_VDW) {
            if (t < c->kappa) { f = c->mon_var[t] == VAR_G ? G : rho; second = 0; }
            else { f = G; second = 1; }
          } else {
            f = rho;
            second = t == 1;
          }
          double s2 = 0.0;
          for (int k = 0; k < d; ++k) {
            int ip[3] = {i0, i1, i2}, im[3] = {i0, i1, i2};
            ip[k] += 1;
            im[k] -= 1;
            double fp = f[pidx(&p1, ip[0], ip[1], ip[2])], fm = f[pidx(&p1, im[0], im[1], im[2])];
            double f0 = f[pidx(&p1, i0, i1, i2)];
            double h = dxi(c, k);
            double g = second ? (fp - 2.0 * f0 + fm) / (h * h) : (fp - fm) / (2.0 * h);
            s2 += g * g;
          }
          double val = c->monitor_kind == MON_VDW ? s2 : sqrt(s2);
          term[t * N + qi] = val;
          if (val > mxv[t] && !solid(c, i0, i1)) mxv[t] = val; /* maxima over the fluid nodes */
        }
      }
  for (long q = 0; q < N; ++q) {
    double s = 1.0;
    for (int t = 0; t < nterm; ++t)
      if (mxv[t] > 0.0) s += c->alpha[t] * term[t * N + q] / mxv[t];
    omega[q] = sqrt(s);
  }
  orc_step_fill_scalar(c, omega);
  free(term);
  free(rho);
  free(G);
  free(rhoi);
  free(Gi);
}

/* low-pass filter, npass passes: omega <- sum_{j in {-1,0,1}^d} (1/2)^(|j|_1 + d) omega_{i+j} */
void orc_filter(const orc_cfg *c, double *omega, int npass) {
  int d = c->dim;
  long N = nodes(c);
  pad_t p1 = make_pad(c, 1);
  double *w = calloc(p1.N, sizeof(double));
  for (int it = 0; it < npass; ++it) {
    to_pad(c, &p1, omega, w);
    fill_ghosts(c, &p1, w, 3, 0);
#pragma omp parallel for collapse(2) schedule(static)
    for (int i2 = 0; i2 < p1.n[2]; ++i2)
      for (int i1 = 0; i1 < p1.n[1]; ++i1)
        for (int i0 = 0; i0 < p1.n[0]; ++i0) {
          double s = 0.0;
          int r2 = d > 2 ? 1 : 0, r1 = d > 1 ? 1 : 0;
          for (int j2 = -r2; j2 <= r2; ++j2)
            for (int j1 = -r1; j1 <= r1; ++j1)
              for (int j0 = -1; j0 <= 1; ++j0) {
                int l1 = abs(j0) + abs(j1) + abs(j2) + d;
                s += ldexp(1.0, -l1) * w[pidx(&p1, i0 + j0, i1 + j1, i2 + j2)];
              }
          omega[iidx(c, i0, i1, i2)] = s;
        }
    orc_step_fill_scalar(c, omega);
  }
  (void)N;
  free(w);
}

/* Jacobi sweeps for the mesh equations (eq. mesh_EL discretised by second-order
 * central differences with omega_{i,k,+-1/2} = (omega_i + omega_{i+-e_k})/2):
 *   x_i <- sum_k (w_{k,+} x_{i+e_k} + w_{k,-} x_{i-e_k})/dxi_k^2 / sum_k (w_{k,+} + w_{k,-})/dxi_k^2.
 * x is updated in place (interior arrays, d fields).  Fixed mode: exactly nsweep sweeps.
 * Tolerance mode (tol > 0): stops after the first sweep whose max update is < tol, or
 * after nsweep sweeps.  Returns the number of sweeps; *resid = max update of the last one. */
int orc_jacobi(const orc_cfg *c, const double *omega, double *x, int nsweep, double tol, double *resid) {
  int d = c->dim;
  long N = nodes(c);
  pad_t p1 = make_pad(c, 1);
  double *w = calloc(p1.N, sizeof(double));
  to_pad(c, &p1, omega, w);
  fill_ghosts(c, &p1, w, 3, 0);
  double *xnew = malloc(sizeof(double) * d * N);
  int it = 0;
  double res = 0.0;
  for (it = 0; it < nsweep;) {
    double **xp = pad_mesh(c, &p1, x, 1);
    res = 0.0;
#pragma omp parallel for collapse(2) reduction(max : res) schedule(static)
    for (int i2 = 0; i2 < p1.n[2]; ++i2)
      for (int i1 = 0; i1 < p1.n[1]; ++i1)
        for (int i0 = 0; i0 < p1.n[0]; ++i0) {
          long qp = pidx(&p1, i0, i1, i2), qi = iidx(c, i0, i1, i2);
          double den = 0.0, num[3] = {0, 0, 0};
          for (int k = 0; k < d; ++k) {
            int ip[3] = {i0, i1, i2}, im[3] = {i0, i1, i2};
            ip[k] += 1;
            im[k] -= 1;
            long qpp = pidx(&p1, ip[0], ip[1], ip[2]), qpm = pidx(&p1, im[0], im[1], im[2]);
            double h2 = dxi(c, k) * dxi(c, k);
            double wp = 0.5 * (w[qp] + w[qpp]), wm = 0.5 * (w[qp] + w[qpm]);
            den += (wp + wm) / h2;
            for (int j = 0; j < d; ++j) num[j] += (wp * xp[j][qpp] + wm * xp[j][qpm]) / h2;
          }
          const int held = solid(c, i0, i1); /* set by the fill below */
          for (int j = 0; j < d; ++j) {
            double v = num[j] / den;
            double u = fabs(v - x[j * N + qi]);
            if (u > res && !held) res = u;
            xnew[j * N + qi] = v;
          }
        }
    free_fields(xp, d);
    memcpy(x, xnew, sizeof(double) * d * N);
    orc_step_fill_mesh(c, x);
    ++it;
    if (tol > 0.0 && res < tol) break;
  }
  if (resid) *resid = res;
  free(w);
  free(xnew);
  return it;
}

/* Red-black successive over-relaxation for the same discrete mesh equations (an alternative
 * to the Jacobi iteration above with the same fixed point; Gauss-Seidel when relax = 1).
 * A sweep is two half-sweeps: first the nodes with i0 + i1 + i2 even, then the odd ones.  In a
 * half-sweep every node of that colour solves its own equation for its own value, the other
 * colour held fixed: at an outflow wall the mirror image of the node is the node itself
 * (normal coordinate 2 wall - x, tangential x), so that term moves to the left-hand side,
 *   normal:     (den + w) x = rest + 2 wall w,     tangential: (den - w) x = rest,
 * and elsewhere the solve is the Jacobi value v.  Then x <- x + relax (v - x).  Periodic
 * directions need an even node count (the wrap would join two nodes of one colour); returns -1
 * then.  Exactly nsweep sweeps; *resid = the largest |v - x| (unrelaxed) of the last sweep.
 * Returns the number of sweeps. */
int orc_sor(const orc_cfg *c, const double *omega, double *x, int nsweep, double relax, double *resid) {
  int d = c->dim;
  long N = nodes(c);
  for (int k = 0; k < d; ++k)
    if (c->bc[k] == BC_PERIODIC && c->n[k] % 2) return -1;
  if (has_step(c)) return -1;
  pad_t p1 = make_pad(c, 1);
  double *w = calloc(p1.N, sizeof(double));
  to_pad(c, &p1, omega, w);
  fill_ghosts(c, &p1, w, 3, 0);
  double res = 0.0;
  for (int it = 0; it < nsweep; ++it) {
    res = 0.0;
    for (int colour = 0; colour < 2; ++colour) {
      double **xp = pad_mesh(c, &p1, x, 1);
      for (int i2 = 0; i2 < p1.n[2]; ++i2)
        for (int i1 = 0; i1 < p1.n[1]; ++i1)
          for (int i0 = 0; i0 < p1.n[0]; ++i0) {
            if ((i0 + i1 + i2) % 2 != colour) continue;
            long qp = pidx(&p1, i0, i1, i2), qi = iidx(c, i0, i1, i2);
            double den[3] = {0, 0, 0}, num[3] = {0, 0, 0};
            for (int k = 0; k < d; ++k) {
              double h2 = dxi(c, k) * dxi(c, k);
              for (int side = 0; side < 2; ++side) {
                int in[3] = {i0, i1, i2};
                in[k] += side ? 1 : -1;
                long qn = pidx(&p1, in[0], in[1], in[2]);
                double wf = 0.5 * (w[qp] + w[qn]) / h2;
                int self = c->bc[k] != BC_PERIODIC && (in[k] < 0 || in[k] >= c->n[k]);
                for (int j = 0; j < d; ++j) {
                  if (!self) {
                    den[j] += wf;
                    num[j] += wf * xp[j][qn];
                  } else if (j == k) {
                    den[j] += 2.0 * wf;
                    num[j] += wf * 2.0 * (side ? c->hi[k] : c->lo[k]);
                  }
                  /* tangential self term: w x on both sides, dropped */
                }
              }
            }
            for (int j = 0; j < d; ++j) {
              double v = num[j] / den[j], old = x[j * N + qi];
              if (fabs(v - old) > res) res = fabs(v - old);
              x[j * N + qi] = old + relax * (v - old);
            }
          }
      free_fields(xp, d);
    }
  }
  if (resid) *resid = res;
  free(w);
  return nsweep;
}

/* movement limiter: Delta_gamma = min(1, min over nodes and directions of the bound
 * -(x_k(i) - x_k(i - e_k))/(2 dx_k) if dx_k < 0, (x_k(i + e_k) - x_k(i))/(2 dx_k) if dx_k > 0),
 * dx = xmu - xn; neighbours from the ghost-extended x^n. */
double orc_limiter(const orc_cfg *c, const double *xn, const double *xmu) {
  int d = c->dim;
  long N = nodes(c);
  pad_t p1 = make_pad(c, 1);
  double **xp = pad_mesh(c, &p1, xn, 1);
  double g = 1.0;
#pragma omp parallel for collapse(2) reduction(min : g) schedule(static)
  for (int i2 = 0; i2 < p1.n[2]; ++i2)
    for (int i1 = 0; i1 < p1.n[1]; ++i1)
      for (int i0 = 0; i0 < p1.n[0]; ++i0) {
        long qi = iidx(c, i0, i1, i2), qp = pidx(&p1, i0, i1, i2);
        if (solid(c, i0, i1)) continue; /* fluid nodes only */
        for (int k = 0; k < d; ++k) {
          double dx = xmu[k * N + qi] - xn[k * N + qi];
          int ip[3] = {i0, i1, i2}, im[3] = {i0, i1, i2};
          ip[k] += 1;
          im[k] -= 1;
          double bnd;
          if (dx < 0.0) bnd = -(xp[k][qp] - xp[k][pidx(&p1, im[0], im[1], im[2])]) / (2.0 * dx);
          else if (dx > 0.0) bnd = (xp[k][pidx(&p1, ip[0], ip[1], ip[2])] - xp[k][qp]) / (2.0 * dx);
          else continue;
          if (bnd < g) g = bnd;
        }
      }
  free_fields(xp, d);
  return g;
}

/* Mesh redistribution between time steps (Section 4): monitor from (U^n) -> filter ->
 * Jacobi from x^[0] = x^n (+ warm_dx) -> limiter -> dt (CFL, or dt_fixed) ->
 * xdot = Delta_gamma (x^[mu] - x^n)/dt.  Outputs: xdot, *dt, *gamma, *resid, *sweeps.
 * omega_out / xmu_out (may be NULL) receive the filtered monitor and x^[mu]. */
void orc_redistribute(const orc_cfg *c, const double *JU, const double *J, const double *xn,
                      const double *warm_dx, double *xdot, double *dt_out, double *gamma_out,
                      double *resid_out, int *sweeps_out, double *omega_out, double *xmu_out) {
  int d = c->dim;
  long N = nodes(c);
  double *omega = malloc(sizeof(double) * N);
  orc_monitor(c, JU, J, omega);
  orc_filter(c, omega, c->n_filter);
  double *xm = malloc(sizeof(double) * d * N);
  for (long q = 0; q < d * N; ++q) xm[q] = xn[q] + (warm_dx ? warm_dx[q] : 0.0);
  double res = 0.0;
  int sw = orc_jacobi(c, omega, xm, c->mu, c->fixed_mu ? 0.0 : c->mesh_tol, &res);
  if (!c->fixed_mu && !(res < c->mesh_tol)) raise_flag(F_NOTCONVERGED);
  double gam = orc_limiter(c, xn, xm);
  double dt = c->dt_fixed > 0.0 ? c->dt_fixed : orc_cfl_dt(c, JU, J, xn);
  for (long q = 0; q < d * N; ++q) xdot[q] = gam * (xm[q] - xn[q]) / dt;
  if (dt_out) *dt_out = dt;
  if (gamma_out) *gamma_out = gam;
  if (resid_out) *resid_out = res;
  if (sweeps_out) *sweeps_out = sw;
  if (omega_out) memcpy(omega_out, omega, sizeof(double) * N);
  if (xmu_out) memcpy(xmu_out, xm, sizeof(double) * d * N);
  free(omega);
  free(xm);
}

/* One full time step in place: redistribute (if moving), three SSP-RK3 stages,
 * x^{n+1} = x^n + dt xdot.  moving = 0 keeps the mesh fixed (uniform-mesh scheme).
 * Returns dt. */
double orc_step(const orc_cfg *c, double *JU, double *J, double *x, int moving) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  double *xdot = calloc((long)d * N, sizeof(double));
  double dt;
  if (moving) {
    orc_redistribute(c, JU, J, x, NULL, xdot, &dt, NULL, NULL, NULL, NULL, NULL);
  } else {
    dt = c->dt_fixed > 0.0 ? c->dt_fixed : orc_cfl_dt(c, JU, J, x);
  }
  double *JU1 = malloc(sizeof(double) * nv * N), *J1 = malloc(sizeof(double) * N);
  double *JU2 = malloc(sizeof(double) * nv * N), *J2 = malloc(sizeof(double) * N);
  const double *xd = moving ? xdot : NULL;
  orc_rk_stage(c, 0, dt, JU, J, JU, J, x, xd, JU1, J1);
  orc_rk_stage(c, 1, dt, JU, J, JU1, J1, x, xd, JU2, J2);
  orc_rk_stage(c, 2, dt, JU, J, JU2, J2, x, xd, JU, J);
  if (moving) {
    for (long q = 0; q < d * N; ++q) x[q] += dt * xdot[q];
    orc_step_fill_mesh(c, x);
  }
  free(JU1);
  free(J1);
  free(JU2);
  free(J2);
  free(xdot);
  return dt;
}

/* JU = J U(prim) at every node; prim = (rho, v_1..v_d, p) fields */
void orc_init_state(const orc_cfg *c, const double *prim, const double *J, double *JU) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  for (long q = 0; q < N; ++q) {
    double pr[NVMAX], U[NVMAX];
    for (int v = 0; v < nv; ++v) pr[v] = prim[v * N + q];
    orc_prim_to_cons(c, pr, U);
    for (int v = 0; v < nv; ++v) JU[v * N + q] = J[q] * U[v];
  }
}

/* total entropy sum_i J_i eta(U_i) * cell volume */
double orc_total_entropy(const orc_cfg *c, const double *JU, const double *J) {
  int d = c->dim, nv = d + 2;
  long N = nodes(c);
  double vol = 1.0, s = 0.0;
  for (int k = 0; k < d; ++k) vol *= dxi(c, k);
  for (long q = 0; q < N; ++q) {
    double U[NVMAX];
    for (int v = 0; v < nv; ++v) U[v] = JU[v * N + q] / J[q];
    s += J[q] * orc_entropy(c, U) * vol;
  }
  return s;
}
