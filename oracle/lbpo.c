/*
 * lbpo.c -- CPU ORACLE (test infrastructure only; see lbpo.h).
 *
 * One time step, written out in the order the method defines it and with no
 * blocking, fusion or reordering:
 *   1. moments        rho = sum f, j = sum e f, T = sum g          (Sec. III.A)
 *   2. EOS and psi    Peng-Robinson p(rho,T), Eq. (56); psi from p
 *   3. force          pseudopotential interaction + buoyancy (Sec. IV.B)
 *   4. velocity       v = (j + F/2)/rho
 *   5. thermal source phi of Eq. (28) (underlined terms) with isotropic
 *                     differences; S0 = phi + 0.5 dt d_t(phi), Eq. (46),
 *                     d_t(phi) taken as a backward difference (Sec. III.B)
 *   6. flow MRT collision with forcing (the cited pseudopotential model)
 *   7. improved thermal MRT collision, Eqs. (45), (46), (53), (54), (55)
 *      (or, for the Gong-Cheng model, the BGK collision of Eq. (12) with
 *      the equilibrium of Eq. (14) and the source of Eq. (13); or, for the
 *      BGK form of the improved model, Eq. (33) with Eqs. (29), (31), (32))
 *   8. streaming, Eq. (47), with the boundary rules below.
 *
 * Every array is a plain [q][ny][nx] (distributions) or [ny][nx] (fields)
 * FP64 array; every sum runs over the lattice directions in the order 0..8.
 *
 * Readings where the paper is silent (each is a named constant or rule here):
 *  - D2Q9 order: 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+1,+1), 6 (-1,+1),
 *    7 (-1,-1), 8 (+1,-1); M is the orthogonal Lallemand-Luo matrix in the
 *    row order (rho, e, eps, jx, qx, jy, qy, pxx, pxy).  With that M,
 *    M times Eq. (29) reproduces Eq. (44).
 *  - Flow model (cited, not printed): MRT with m^eq = rho(1, -2+3v^2,
 *    1-3v^2, vx, -vx, vy, -vy, vx^2-vy^2, vx vy), forcing source S_f in
 *    moment space with the sigma-term on moments 1 and 2, collision
 *    m* = m - S(m - m^eq) + (I - S/2) S_f, v = (j + F/2)/rho.
 *  - psi = sqrt(2 (p_EOS - rho c_s^2) / (G c^2)), G < 0; interaction force
 *    F_m = -G psi(x) sum_a w_a psi(x+e_a) e_a with w = 1/3 (axis), 1/12 (diag).
 *  - Isotropic differences: d_i X = (1/c_s^2) sum_a w_a X(x+e_a) e_ai,
 *    lap X = (2/c_s^2) sum_a w_a (X(x+e_a) - X(x)).
 *  - k = (1/s_g3 - 1/2) c_s^2 dt (Eq. A13/A22) in the -div(k grad T) term.
 *  - First step: phi(t-dt) := phi(t), so d_t(phi) = 0.
 *  - Boundaries.  A neighbour outside the lattice is first wrapped on
 *    periodic sides; if it is still outside it is a ghost that takes rho and
 *    psi from the nearest lattice node (coordinates clamped), v = 0 at a
 *    wall and v of that node at an open side, and T = the temperature of
 *    the crossed side (the y side when both are crossed; the y- wall carries
 *    T_hot on its hot-spot columns).  Streaming from a ghost: across a wall,
 *    halfway bounce-back f_a(x) = f*_abar(x) and anti-bounce-back
 *    g_a(x) = -g*_abar(x) + 2 wg_a T_ghost; across an open side,
 *    f_a(x) = f*_a(clamped source) and g_a(x) = wg_a T_ghost.  Here wg is the
 *    rest equilibrium of Eq. (53), wg = M^-1 (1,-2,2,0,...,0), or, for the
 *    BGK models, that of Eq. (14) / Eq. (29), wg = omega.  A wall wins over an
 *    open side at corners.
 *  - Wetting (a reading: the paper states contact angles, Sec. IV.A and
 *    IV.B, but defines no wetting scheme).  In the interaction force only, a
 *    ghost across a wall has psi(rho_w, T_n), rho_w = (1 + wet_amp) rho_n -
 *    wet_shift clamped to [0, 0.9/b], where n is the nearest lattice node: a
 *    virtual solid density taken from the adjacent fluid.  wet_amp =
 *    wet_shift = 0 is psi_n, the neutral rule above.
 *  - Gong-Cheng model: v in Eq. (14) is the flow velocity of step 4, and the
 *    divergence of Eq. (13) uses the same isotropic differences.
 *  - BGK form of the improved model: d_t(T v) of Eq. (31) is the backward
 *    difference T v(t) - T v(t - dt) (zero on the first step, as d_t phi),
 *    and G_a + (dt/2) d_t G_a of Eq. (32) is omega_a S0 with S0 of step 5.
 *  - rho_ave of the buoyancy force is the mean initial density.
 */
#include "lbpo.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define Q 9
#define CS2 (1.0 / 3.0)

static const int EX[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
static const int EY[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
static const int OPP[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};
/* lattice weights omega_a of the D2Q9 set (Sec. II.B) */
static const double WL[Q] = {4.0 / 9.0,  1.0 / 9.0,  1.0 / 9.0,
                             1.0 / 9.0,  1.0 / 9.0,  1.0 / 36.0,
                             1.0 / 36.0, 1.0 / 36.0, 1.0 / 36.0};
/* pseudopotential force weights w(|e|^2): 1/3 axis, 1/12 diagonal */
static const double WF[Q] = {0.0,        1.0 / 3.0,  1.0 / 3.0,
                             1.0 / 3.0,  1.0 / 3.0,  1.0 / 12.0,
                             1.0 / 12.0, 1.0 / 12.0, 1.0 / 12.0};
/* orthogonal transformation matrix of the MRT operator (Eq. 42) */
static const double MM[Q][Q] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1},         /* rho */
    {-4, -1, -1, -1, -1, 2, 2, 2, 2},    /* e   */
    {4, -2, -2, -2, -2, 1, 1, 1, 1},     /* eps */
    {0, 1, 0, -1, 0, 1, -1, -1, 1},      /* jx  */
    {0, -2, 0, 2, 0, 1, -1, -1, 1},      /* qx  */
    {0, 0, 1, 0, -1, 1, 1, -1, -1},      /* jy  */
    {0, 0, -2, 0, 2, 1, 1, -1, -1},      /* qy  */
    {0, 1, -1, 1, -1, 0, 0, 0, 0},       /* pxx */
    {0, 0, 0, 0, 0, 1, -1, 1, -1}};      /* pxy */

enum { G_INSIDE = 0, G_WALL = 1, G_OPEN = 2 };

struct lbpo_handle {
  lbpo_config c;
  int nx, ny;
  size_t n;
  double Minv[Q][Q];
  double wg[Q];        /* rest equilibrium of Eq. (53) per unit T */
  double Tc, kappa, k_th;
  double *f, *g;       /* f(t), g(t) */
  double *fp, *gp;     /* post-collision f*, g* */
  double *rho, *jx, *jy, *T, *psi, *Fx, *Fy, *ux, *uy;
  double *phi, *phi_prev, *S0;
  double *tvx_prev, *tvy_prev; /* T v of the previous step (BGK form) */
  int phi_valid;
  int initialised;
  int bad;
  double rho_ave;
  int64_t step;
  double last_sum_S0, last_sum_Fx, last_sum_Fy;
};

/* ------------------------------------------------------------------ EOS -- */

double lbpo_Tc(double a, double b, double R) {
  /* a = 0.45724 R^2 Tc^2 / pc and b = 0.0778 R Tc / pc (Eq. 56) give
     a / b = (0.45724 / 0.0778) R Tc */
  return 0.0778 * a / (0.45724 * b * R);
}

static double pr_kappa(double omega) {
  return 0.37464 + 1.54226 * omega - 0.26992 * omega * omega;
}

/* vartheta(T) of Eq. (56) */
static double pr_theta(double kappa, double Tc, double T) {
  double s = 1.0 + kappa * (1.0 - sqrt(T / Tc));
  return s * s;
}

/* d vartheta / dT */
static double pr_dtheta(double kappa, double Tc, double T) {
  double s = 1.0 + kappa * (1.0 - sqrt(T / Tc));
  return 2.0 * s * (-kappa) * (0.5 / sqrt(T * Tc));
}

double lbpo_p_eos(const lbpo_config *c, double rho, double T) {
  double Tc = lbpo_Tc(c->a, c->b, c->R);
  double th = pr_theta(pr_kappa(c->omega), Tc, T);
  return rho * c->R * T / (1.0 - c->b * rho) -
         c->a * th * rho * rho /
             (1.0 + 2.0 * c->b * rho - c->b * c->b * rho * rho);
}

/* (d p_EOS / d T) at constant rho */
double lbpo_dpdT(const lbpo_config *c, double rho, double T) {
  double Tc = lbpo_Tc(c->a, c->b, c->R);
  double dth = pr_dtheta(pr_kappa(c->omega), Tc, T);
  return rho * c->R / (1.0 - c->b * rho) -
         c->a * dth * rho * rho /
             (1.0 + 2.0 * c->b * rho - c->b * c->b * rho * rho);
}

/* --------------------------------------------------------- MRT pieces -- */

void lbpo_matrix_M(double out[81]) {
  for (int k = 0; k < Q; ++k)
    for (int a = 0; a < Q; ++a) out[k * Q + a] = MM[k][a];
}

/* M is orthogonal (rows mutually orthogonal), so M^-1 = M^T diag(1/|row|^2) */
static void build_Minv(double Minv[Q][Q]) {
  for (int k = 0; k < Q; ++k) {
    double nrm = 0.0;
    for (int a = 0; a < Q; ++a) nrm += MM[k][a] * MM[k][a];
    for (int a = 0; a < Q; ++a) Minv[a][k] = MM[k][a] / nrm;
  }
}

void lbpo_matrix_Minv(double out[81]) {
  double Mi[Q][Q];
  build_Minv(Mi);
  for (int a = 0; a < Q; ++a)
    for (int k = 0; k < Q; ++k) out[a * Q + k] = Mi[a][k];
}

/* flow equilibria in moment space (the cited pseudopotential MRT model) */
void lbpo_flow_meq(double rho, double vx, double vy, double out[9]) {
  double v2 = vx * vx + vy * vy;
  out[0] = rho;
  out[1] = rho * (-2.0 + 3.0 * v2);
  out[2] = rho * (1.0 - 3.0 * v2);
  out[3] = rho * vx;
  out[4] = -rho * vx;
  out[5] = rho * vy;
  out[6] = -rho * vy;
  out[7] = rho * (vx * vx - vy * vy);
  out[8] = rho * vx * vy;
}

/* thermal equilibria in moment space, Eq. (53): m1^eq + m2^eq = 0 */
void lbpo_thermal_meq(double T, double vx, double vy, double out[9]) {
  out[0] = T;
  out[1] = -2.0 * T;
  out[2] = 2.0 * T;
  out[3] = T * vx;
  out[4] = -T * vx;
  out[5] = T * vy;
  out[6] = -T * vy;
  out[7] = 0.0;
  out[8] = 0.0;
}

static void mat_vec(const double A[Q][Q], const double *x, double *y) {
  for (int k = 0; k < Q; ++k) {
    double s = 0.0;
    for (int a = 0; a < Q; ++a) s += A[k][a] * x[a];
    y[k] = s;
  }
}

/* D2Q9 equilibrium of Eq. (14):
 * omega_a T [1 + e.v/c_s^2 + (e.v)^2/(2 c_s^4) - v.v/(2 c_s^2)] */
void lbpo_gc_geq(double T, double vx, double vy, double out[9]) {
  double v2 = vx * vx + vy * vy;
  for (int a = 0; a < Q; ++a) {
    double eu = EX[a] * vx + EY[a] * vy;
    out[a] = WL[a] * T *
             (1.0 + eu / CS2 + eu * eu / (2.0 * CS2 * CS2) - v2 / (2.0 * CS2));
  }
}

/* D2Q9 equilibrium of Eq. (29): omega_a T (1 + e.v / c_s^2) */
void lbpo_lin_geq(double T, double vx, double vy, double out[9]) {
  for (int a = 0; a < Q; ++a)
    out[a] = WL[a] * T * (1.0 + (EX[a] * vx + EY[a] * vy) / CS2);
}

/* ------------------------------------------------------- boundaries -- */

typedef struct {
  int kind;   /* G_INSIDE, G_WALL or G_OPEN */
  size_t idx; /* lattice node after wrapping (inside) or clamping (ghost) */
  double T;   /* ghost temperature (unused when inside) */
} ghost_t;

static double side_T(const lbpo_handle *h, int side, int col) {
  if (side == 2 && col >= h->c.hot_x0 && col < h->c.hot_x1) return h->c.T_hot;
  return h->c.T_bc[side];
}

static ghost_t resolve(const lbpo_handle *h, int x, int y) {
  ghost_t gh;
  int xs = -1, ys = -1;
  if (x < 0 || x >= h->nx) {
    int side = x < 0 ? 0 : 1;
    if (h->c.bc[side] == LBPO_BC_PERIODIC) {
      x = (x + h->nx) % h->nx;
    } else {
      xs = side;
      x = x < 0 ? 0 : h->nx - 1;
    }
  }
  if (y < 0 || y >= h->ny) {
    int side = y < 0 ? 2 : 3;
    if (h->c.bc[side] == LBPO_BC_PERIODIC) {
      y = (y + h->ny) % h->ny;
    } else {
      ys = side;
      y = y < 0 ? 0 : h->ny - 1;
    }
  }
  gh.idx = (size_t)y * (size_t)h->nx + (size_t)x;
  gh.T = 0.0;
  if (xs < 0 && ys < 0) {
    gh.kind = G_INSIDE;
  } else {
    if ((ys >= 0 && h->c.bc[ys] == LBPO_BC_WALL) ||
        (xs >= 0 && h->c.bc[xs] == LBPO_BC_WALL))
      gh.kind = G_WALL;
    else
      gh.kind = G_OPEN;
    gh.T = ys >= 0 ? side_T(h, ys, x) : side_T(h, xs, x);
  }
  return gh;
}

/* stencil values of the fields at a (possibly ghost) neighbour */
static double nb_rho(const lbpo_handle *h, ghost_t gh) { return h->rho[gh.idx]; }
/* psi of a neighbour in the interaction force; across a wall, that of the
 * virtual density of the wetting reading */
static double nb_psi(const lbpo_handle *h, ghost_t gh) {
  const lbpo_config *c = &h->c;
  if (gh.kind != G_WALL || (c->wet_amp == 0.0 && c->wet_shift == 0.0))
    return h->psi[gh.idx];
  double rw = (1.0 + c->wet_amp) * h->rho[gh.idx] - c->wet_shift;
  if (rw < 0.0) rw = 0.0;
  if (rw > 0.9 / c->b) rw = 0.9 / c->b;
  double psi2 = 2.0 * (lbpo_p_eos(c, rw, h->T[gh.idx]) - rw * CS2) / c->G;
  return sqrt(psi2 > 0.0 ? psi2 : 0.0);
}
static double nb_T(const lbpo_handle *h, ghost_t gh) {
  return gh.kind == G_INSIDE ? h->T[gh.idx] : gh.T;
}
static double nb_ux(const lbpo_handle *h, ghost_t gh) {
  return gh.kind == G_WALL ? 0.0 : h->ux[gh.idx];
}
static double nb_uy(const lbpo_handle *h, ghost_t gh) {
  return gh.kind == G_WALL ? 0.0 : h->uy[gh.idx];
}

/* --------------------------------------------------------- lifecycle -- */

static int check_config(const lbpo_config *c) {
  if (c->nx < 4 || c->ny < 4) return LBPO_ERR_ARG;
  if ((c->bc[0] == LBPO_BC_PERIODIC) != (c->bc[1] == LBPO_BC_PERIODIC))
    return LBPO_ERR_ARG;
  if ((c->bc[2] == LBPO_BC_PERIODIC) != (c->bc[3] == LBPO_BC_PERIODIC))
    return LBPO_ERR_ARG;
  for (int i = 0; i < 4; ++i)
    if (c->bc[i] < 0 || c->bc[i] > 2) return LBPO_ERR_ARG;
  if (!isfinite(c->wet_amp) || !(c->wet_amp > -1.0) || !isfinite(c->wet_shift))
    return LBPO_ERR_ARG;
  for (int i = 0; i < Q; ++i) {
    if (!(c->s_f[i] > 0.0 && c->s_f[i] < 2.0)) return LBPO_ERR_ARG;
    if (!(c->s_g[i] > 0.0 && c->s_g[i] < 2.0)) return LBPO_ERR_ARG;
  }
  if (!(c->G < 0.0) || !(c->a > 0.0) || !(c->b > 0.0) || !(c->R > 0.0) ||
      !(c->cv > 0.0))
    return LBPO_ERR_ARG;
  if (c->lambda_mode != LBPO_LAMBDA_CONST &&
      c->lambda_mode != LBPO_LAMBDA_RHO_CV_CHI)
    return LBPO_ERR_ARG;
  if (c->thermal_model != LBPO_THERMAL_IMPROVED &&
      c->thermal_model != LBPO_THERMAL_COMPROMISED &&
      c->thermal_model != LBPO_THERMAL_GONG_CHENG &&
      c->thermal_model != LBPO_THERMAL_IMPROVED_BGK)
    return LBPO_ERR_ARG;
  if (c->thermal_model == LBPO_THERMAL_GONG_CHENG &&
      !(c->lambda_mode == LBPO_LAMBDA_CONST ? c->lambda0 > 0.0 : c->chi > 0.0))
    return LBPO_ERR_ARG;
  return LBPO_OK;
}

int lbpo_create(const lbpo_config *cfg, lbpo_handle **out) {
  if (!cfg || !out) return LBPO_ERR_ARG;
  *out = NULL;
  int st = check_config(cfg);
  if (st != LBPO_OK) return st;
  lbpo_handle *h = (lbpo_handle *)calloc(1, sizeof(*h));
  if (!h) return LBPO_ERR_OOM;
  h->c = *cfg;
  h->nx = cfg->nx;
  h->ny = cfg->ny;
  h->n = (size_t)cfg->nx * (size_t)cfg->ny;
  build_Minv(h->Minv);
  if (cfg->thermal_model == LBPO_THERMAL_GONG_CHENG ||
      cfg->thermal_model == LBPO_THERMAL_IMPROVED_BGK) {
    lbpo_gc_geq(1.0, 0.0, 0.0, h->wg);
  } else {
    double meq[Q];
    lbpo_thermal_meq(1.0, 0.0, 0.0, meq);
    mat_vec((const double(*)[Q])h->Minv, meq, h->wg);
  }
  h->Tc = lbpo_Tc(cfg->a, cfg->b, cfg->R);
  h->kappa = pr_kappa(cfg->omega);
  h->k_th = (1.0 / cfg->s_g[3] - 0.5) * CS2;
  size_t n = h->n;
  h->f = (double *)calloc(Q * n, sizeof(double));
  h->g = (double *)calloc(Q * n, sizeof(double));
  h->fp = (double *)calloc(Q * n, sizeof(double));
  h->gp = (double *)calloc(Q * n, sizeof(double));
  double **fields[] = {&h->rho, &h->jx, &h->jy, &h->T,   &h->psi,
                       &h->Fx,  &h->Fy, &h->ux, &h->uy,  &h->phi,
                       &h->phi_prev, &h->S0, &h->tvx_prev, &h->tvy_prev};
  int ok = h->f && h->g && h->fp && h->gp;
  for (size_t i = 0; i < sizeof(fields) / sizeof(fields[0]); ++i) {
    *fields[i] = (double *)calloc(n, sizeof(double));
    ok = ok && *fields[i];
  }
  if (!ok) {
    lbpo_destroy(h);
    return LBPO_ERR_OOM;
  }
  *out = h;
  return LBPO_OK;
}

void lbpo_destroy(lbpo_handle *h) {
  if (!h) return;
  free(h->f); free(h->g); free(h->fp); free(h->gp);
  free(h->rho); free(h->jx); free(h->jy); free(h->T); free(h->psi);
  free(h->Fx); free(h->Fy); free(h->ux); free(h->uy);
  free(h->phi); free(h->phi_prev); free(h->S0);
  free(h->tvx_prev); free(h->tvy_prev);
  free(h);
}

int lbpo_init_fields(lbpo_handle *h, const double *rho, const double *ux,
                     const double *uy, const double *T) {
  if (!h || !rho || !ux || !uy || !T) return LBPO_ERR_ARG;
  for (size_t i = 0; i < h->n; ++i) {
    if (!(rho[i] > 0.0 && rho[i] < 1.0 / h->c.b)) return LBPO_ERR_ARG;
    if (!(T[i] > 0.0) || !isfinite(ux[i]) || !isfinite(uy[i]))
      return LBPO_ERR_ARG;
    double psi2 = 2.0 * (lbpo_p_eos(&h->c, rho[i], T[i]) - rho[i] * CS2) /
                  h->c.G;
    if (!(psi2 >= 0.0)) return LBPO_ERR_ARG;
  }
  double sum = 0.0;
  for (size_t i = 0; i < h->n; ++i) {
    double meq[Q], feq[Q];
    lbpo_flow_meq(rho[i], ux[i], uy[i], meq);
    mat_vec((const double(*)[Q])h->Minv, meq, feq);
    for (int a = 0; a < Q; ++a) h->f[a * h->n + i] = feq[a];
    if (h->c.thermal_model == LBPO_THERMAL_GONG_CHENG) {
      lbpo_gc_geq(T[i], ux[i], uy[i], feq);
    } else if (h->c.thermal_model == LBPO_THERMAL_IMPROVED_BGK) {
      lbpo_lin_geq(T[i], ux[i], uy[i], feq);
    } else {
      lbpo_thermal_meq(T[i], ux[i], uy[i], meq);
      mat_vec((const double(*)[Q])h->Minv, meq, feq);
    }
    for (int a = 0; a < Q; ++a) h->g[a * h->n + i] = feq[a];
    sum += rho[i];
  }
  h->rho_ave = sum / (double)h->n;
  h->phi_valid = 0;
  h->step = 0;
  h->bad = 0;
  h->initialised = 1;
  return LBPO_OK;
}

/* ------------------------------------------------------ the time step -- */

/* steps 1-4: rho, j, T, psi, F, v at every node from f(t), g(t) */
static void macro(lbpo_handle *h) {
  const size_t n = h->n;
  const lbpo_config *c = &h->c;
  for (size_t i = 0; i < n; ++i) {
    double r = 0.0, jx = 0.0, jy = 0.0, T = 0.0;
    for (int a = 0; a < Q; ++a) {
      double fa = h->f[a * n + i];
      r += fa;
      jx += EX[a] * fa;
      jy += EY[a] * fa;
      T += h->g[a * n + i];
    }
    h->rho[i] = r;
    h->jx[i] = jx;
    h->jy[i] = jy;
    h->T[i] = T;
    double p = lbpo_p_eos(c, r, T);
    double psi2 = 2.0 * (p - r * CS2) / c->G; /* c = 1 */
    if (!(psi2 >= 0.0) || !(r > 0.0) || !(r < 1.0 / c->b) || !isfinite(T))
      h->bad = 1;
    h->psi[i] = sqrt(psi2 > 0.0 ? psi2 : 0.0);
  }
  const int freeze = (c->flags & LBPO_FLAG_FREEZE_FLOW) != 0;
  for (int y = 0; y < h->ny; ++y) {
    for (int x = 0; x < h->nx; ++x) {
      size_t i = (size_t)y * h->nx + x;
      double sx = 0.0, sy = 0.0;
      for (int a = 1; a < Q; ++a) {
        ghost_t gh = resolve(h, x + EX[a], y + EY[a]);
        double pn = nb_psi(h, gh);
        sx += WF[a] * pn * EX[a];
        sy += WF[a] * pn * EY[a];
      }
      double Fx = -c->G * h->psi[i] * sx;
      double Fy = -c->G * h->psi[i] * sy;
      Fx += (h->rho[i] - h->rho_ave) * c->gx;
      Fy += (h->rho[i] - h->rho_ave) * c->gy;
      if (freeze) {
        Fx = 0.0;
        Fy = 0.0;
      }
      h->Fx[i] = Fx;
      h->Fy[i] = Fy;
      h->ux[i] = (h->jx[i] + 0.5 * Fx) / h->rho[i];
      h->uy[i] = (h->jy[i] + 0.5 * Fy) / h->rho[i];
    }
  }
}

/* the interaction part of the force alone (for the sigma term) */
static void interaction_force(const lbpo_handle *h, int x, int y, double *Fx,
                              double *Fy) {
  size_t i = (size_t)y * h->nx + x;
  double sx = 0.0, sy = 0.0;
  for (int a = 1; a < Q; ++a) {
    ghost_t gh = resolve(h, x + EX[a], y + EY[a]);
    double pn = nb_psi(h, gh);
    sx += WF[a] * pn * EX[a];
    sy += WF[a] * pn * EY[a];
  }
  *Fx = -h->c.G * h->psi[i] * sx;
  *Fy = -h->c.G * h->psi[i] * sy;
}

/* step 5: phi of Eq. (28) (underlined terms) at node (x, y); for the
 * Gong-Cheng model phi of Eq. (13) */
static double thermal_source(const lbpo_handle *h, int x, int y) {
  const lbpo_config *c = &h->c;
  size_t i = (size_t)y * h->nx + x;
  double dTx = 0.0, dTy = 0.0, lapT = 0.0, drx = 0.0, dry = 0.0;
  double dvx = 0.0, dvy = 0.0;
  for (int a = 1; a < Q; ++a) {
    ghost_t gh = resolve(h, x + EX[a], y + EY[a]);
    double Tn = nb_T(h, gh);
    double rn = nb_rho(h, gh);
    dTx += WL[a] * Tn * EX[a];
    dTy += WL[a] * Tn * EY[a];
    lapT += WL[a] * (Tn - h->T[i]);
    drx += WL[a] * rn * EX[a];
    dry += WL[a] * rn * EY[a];
    dvx += WL[a] * nb_ux(h, gh) * EX[a];
    dvy += WL[a] * nb_uy(h, gh) * EY[a];
  }
  dTx /= CS2;
  dTy /= CS2;
  lapT *= 2.0 / CS2;
  drx /= CS2;
  dry /= CS2;
  double divv = (dvx + dvy) / CS2;
  double rho = h->rho[i], T = h->T[i];
  double lam, dlam_x, dlam_y;
  if (c->lambda_mode == LBPO_LAMBDA_CONST) {
    lam = c->lambda0;
    dlam_x = 0.0;
    dlam_y = 0.0;
  } else {
    lam = rho * c->cv * c->chi;
    dlam_x = c->cv * c->chi * drx;
    dlam_y = c->cv * c->chi * dry;
  }
  double rcv = rho * c->cv;
  if (c->thermal_model == LBPO_THERMAL_GONG_CHENG)
    return T * (1.0 - lbpo_dpdT(c, rho, T) / rcv) * divv;
  /* div(lambda grad T) = lambda lap T + grad lambda . grad T */
  double div_lam_gradT = lam * lapT + (dlam_x * dTx + dlam_y * dTy);
  return div_lam_gradT / rcv - h->k_th * lapT +
         T * (1.0 - lbpo_dpdT(c, rho, T) / rcv) * divv;
}

/* resolve the pulled value of direction a at fluid node (x, y) */
static void stream_node(lbpo_handle *h, int x, int y) {
  const size_t n = h->n;
  size_t i = (size_t)y * h->nx + x;
  const int freeze = (h->c.flags & LBPO_FLAG_FREEZE_FLOW) != 0;
  const int freeze_g = (h->c.flags & LBPO_FLAG_FREEZE_THERMAL) != 0;
  for (int a = 0; a < Q; ++a) {
    ghost_t gh = resolve(h, x - EX[a], y - EY[a]);
    double fn, gn;
    if (gh.kind == G_INSIDE) {
      fn = h->fp[a * n + gh.idx];
      gn = h->gp[a * n + gh.idx];
    } else if (gh.kind == G_WALL) {
      fn = h->fp[OPP[a] * n + i];
      gn = -h->gp[OPP[a] * n + i] + 2.0 * h->wg[a] * gh.T;
    } else {
      fn = h->fp[a * n + gh.idx];
      gn = h->wg[a] * gh.T;
    }
    if (!freeze) h->f[a * n + i] = fn;
    if (!freeze_g) h->g[a * n + i] = gn;
  }
}

static int one_step(lbpo_handle *h) {
  const size_t n = h->n;
  const lbpo_config *c = &h->c;
  const int freeze = (c->flags & LBPO_FLAG_FREEZE_FLOW) != 0;
  macro(h);
  if (h->bad) return LBPO_ERR_NUMERIC;

  /* step 5: thermal source and its discrete-effect correction */
  double sum_S0 = 0.0, sum_Fx = 0.0, sum_Fy = 0.0;
  for (int y = 0; y < h->ny; ++y)
    for (int x = 0; x < h->nx; ++x) {
      size_t i = (size_t)y * h->nx + x;
      h->phi[i] = thermal_source(h, x, y);
    }
  for (size_t i = 0; i < n; ++i) {
    double prev = h->phi_valid ? h->phi_prev[i] : h->phi[i];
    if (c->thermal_model == LBPO_THERMAL_IMPROVED ||
        c->thermal_model == LBPO_THERMAL_IMPROVED_BGK)
      h->S0[i] = h->phi[i] + 0.5 * (h->phi[i] - prev); /* Eqs. (46), (32) */
    else
      h->S0[i] = h->phi[i];
    sum_S0 += h->S0[i];
    sum_Fx += h->Fx[i];
    sum_Fy += h->Fy[i];
  }

  for (int y = 0; y < h->ny; ++y) {
    for (int x = 0; x < h->nx; ++x) {
      size_t i = (size_t)y * h->nx + x;
      double rho = h->rho[i], vx = h->ux[i], vy = h->uy[i], T = h->T[i];
      double m[Q], meq[Q], ms[Q], fa[Q];

      /* step 6: flow MRT collision with the forcing source */
      if (!freeze) {
        for (int a = 0; a < Q; ++a) fa[a] = h->f[a * n + i];
        mat_vec(MM, fa, m);
        lbpo_flow_meq(rho, vx, vy, meq);
        double Fx = h->Fx[i], Fy = h->Fy[i], Fmx, Fmy;
        interaction_force(h, x, y, &Fmx, &Fmy);
        double psi2 = h->psi[i] * h->psi[i];
        double Fm2 = Fmx * Fmx + Fmy * Fmy;
        double vF = vx * Fx + vy * Fy;
        double S[Q];
        S[0] = 0.0;
        S[1] = 6.0 * vF +
               12.0 * c->sigma * Fm2 / (psi2 * (1.0 / c->s_f[1] - 0.5));
        S[2] = -6.0 * vF -
               12.0 * c->sigma * Fm2 / (psi2 * (1.0 / c->s_f[2] - 0.5));
        S[3] = Fx;
        S[4] = -Fx;
        S[5] = Fy;
        S[6] = -Fy;
        S[7] = 2.0 * (vx * Fx - vy * Fy);
        S[8] = vx * Fy + vy * Fx;
        for (int k = 0; k < Q; ++k)
          ms[k] = m[k] - c->s_f[k] * (m[k] - meq[k]) +
                  (1.0 - 0.5 * c->s_f[k]) * S[k];
        mat_vec((const double(*)[Q])h->Minv, ms, fa);
        for (int a = 0; a < Q; ++a) h->fp[a * n + i] = fa[a];
      }

      if (c->thermal_model == LBPO_THERMAL_GONG_CHENG) {
        /* step 7 of the Gong-Cheng model: Eq. (12) with G_a = omega_a phi,
         * g^eq of Eq. (14) and chi = lambda/(rho c_V) = (tau_g - 1/2) c_s^2 */
        double lam = c->lambda_mode == LBPO_LAMBDA_CONST ? c->lambda0
                                                         : rho * c->cv * c->chi;
        double tau = lam / (rho * c->cv * CS2) + 0.5;
        double geq[Q];
        lbpo_gc_geq(T, vx, vy, geq);
        for (int a = 0; a < Q; ++a) {
          double ga = h->g[a * n + i];
          h->gp[a * n + i] = ga - (ga - geq[a]) / tau + WL[a] * h->phi[i];
        }
        continue;
      }

      if (c->thermal_model == LBPO_THERMAL_IMPROVED_BGK) {
        /* step 7 of the BGK form, Eq. (33): BGK relaxation towards Eq. (29),
         * source G + (dt/2) d_t G = omega_a S0 (Eq. 32) and the correction
         * C_a = (1 - 1/(2 tau)) omega_a e_a . d_t(T v) / c_s^2 (Eq. 31) */
        double tau = 1.0 / c->s_g[3];
        double dtx = 0.0, dty = 0.0;
        if (h->phi_valid) {
          dtx = T * vx - h->tvx_prev[i];
          dty = T * vy - h->tvy_prev[i];
        }
        double geq[Q];
        lbpo_lin_geq(T, vx, vy, geq);
        for (int a = 0; a < Q; ++a) {
          double ga = h->g[a * n + i];
          double Ca = (1.0 - 0.5 / tau) * WL[a] *
                      (EX[a] * dtx + EY[a] * dty) / CS2;
          h->gp[a * n + i] =
              ga - (ga - geq[a]) / tau + WL[a] * h->S0[i] + Ca;
        }
        continue;
      }

      /* step 7: improved thermal MRT collision */
      for (int a = 0; a < Q; ++a) fa[a] = h->g[a * n + i];
      mat_vec(MM, fa, m);
      lbpo_thermal_meq(T, vx, vy, meq);               /* Eq. (53) */
      for (int k = 0; k < Q; ++k)                     /* Eq. (45) */
        ms[k] = m[k] - c->s_g[k] * (m[k] - meq[k]);
      ms[0] += h->S0[i];                              /* Eq. (46) */
      if (c->thermal_model == LBPO_THERMAL_IMPROVED) { /* Eqs. (54)-(55) */
        ms[3] += (1.0 - 0.5 * c->s_g[3]) * c->s_g[4] * (m[4] - meq[4]);
        ms[5] += (1.0 - 0.5 * c->s_g[5]) * c->s_g[6] * (m[6] - meq[6]);
      }
      mat_vec((const double(*)[Q])h->Minv, ms, fa);
      for (int a = 0; a < Q; ++a) h->gp[a * n + i] = fa[a];
    }
  }

  /* step 8: streaming, Eq. (47) */
  for (int y = 0; y < h->ny; ++y)
    for (int x = 0; x < h->nx; ++x) stream_node(h, x, y);

  memcpy(h->phi_prev, h->phi, n * sizeof(double));
  if (c->thermal_model == LBPO_THERMAL_IMPROVED_BGK)
    for (size_t i = 0; i < n; ++i) {
      h->tvx_prev[i] = h->T[i] * h->ux[i];
      h->tvy_prev[i] = h->T[i] * h->uy[i];
    }
  h->phi_valid = 1;
  h->last_sum_S0 = sum_S0;
  h->last_sum_Fx = sum_Fx;
  h->last_sum_Fy = sum_Fy;
  h->step += 1;
  return LBPO_OK;
}

int lbpo_step(lbpo_handle *h, int64_t nsteps) {
  if (!h || nsteps < 0) return LBPO_ERR_ARG;
  if (!h->initialised) return LBPO_ERR_STATE;
  for (int64_t s = 0; s < nsteps; ++s) {
    int st = one_step(h);
    if (st != LBPO_OK) return st;
  }
  return LBPO_OK;
}

int lbpo_get_rho_u_T(lbpo_handle *h, double *rho, double *ux, double *uy,
                     double *T) {
  if (!h) return LBPO_ERR_ARG;
  if (!h->initialised) return LBPO_ERR_STATE;
  macro(h);
  size_t bytes = h->n * sizeof(double);
  if (rho) memcpy(rho, h->rho, bytes);
  if (ux) memcpy(ux, h->ux, bytes);
  if (uy) memcpy(uy, h->uy, bytes);
  if (T) memcpy(T, h->T, bytes);
  return h->bad ? LBPO_ERR_NUMERIC : LBPO_OK;
}

int lbpo_get_field(lbpo_handle *h, int field, double *out) {
  if (!h || !out) return LBPO_ERR_ARG;
  if (!h->initialised) return LBPO_ERR_STATE;
  macro(h);
  const double *src = NULL;
  switch (field) {
    case LBPO_FIELD_RHO: src = h->rho; break;
    case LBPO_FIELD_T: src = h->T; break;
    case LBPO_FIELD_UX: src = h->ux; break;
    case LBPO_FIELD_UY: src = h->uy; break;
    case LBPO_FIELD_PSI: src = h->psi; break;
    case LBPO_FIELD_FX: src = h->Fx; break;
    case LBPO_FIELD_FY: src = h->Fy; break;
    case LBPO_FIELD_PHI_PREV: src = h->phi_prev; break;
    case LBPO_FIELD_JX: src = h->jx; break;
    case LBPO_FIELD_JY: src = h->jy; break;
    default: return LBPO_ERR_ARG;
  }
  memcpy(out, src, h->n * sizeof(double));
  return LBPO_OK;
}

int lbpo_get_diag(lbpo_handle *h, lbpo_diag *d) {
  if (!h || !d) return LBPO_ERR_ARG;
  if (!h->initialised) return LBPO_ERR_STATE;
  macro(h);
  memset(d, 0, sizeof(*d));
  double half = 0.5 * (h->c.rho_l + h->c.rho_v);
  double count = 0.0;
  for (size_t i = 0; i < h->n; ++i) {
    double r = h->rho[i];
    d->mass += r;
    d->sum_T += h->T[i];
    d->sum_rhocvT += r * h->c.cv * h->T[i];
    double frac = (r - h->c.rho_v) / (h->c.rho_l - h->c.rho_v);
    if (frac < 0.0) frac = 0.0;
    if (frac > 1.0) frac = 1.0;
    d->liquid_area += frac;
    if (r > half) count += 1.0;
    double sp = sqrt(h->ux[i] * h->ux[i] + h->uy[i] * h->uy[i]);
    if (sp > d->max_speed) d->max_speed = sp;
    if (!isfinite(r) || !isfinite(h->T[i])) d->nonfinite = 1;
  }
  if (h->bad) d->nonfinite = 1;
  d->radius = sqrt(d->liquid_area / M_PI);
  d->radius_count = sqrt(count / M_PI);
  d->sum_S0 = h->last_sum_S0;
  d->sum_Fx = h->last_sum_Fx;
  d->sum_Fy = h->last_sum_Fy;
  d->step = h->step;
  return LBPO_OK;
}

int lbpo_get_state(lbpo_handle *h, double *f, double *g, double *phi_prev,
                   int32_t *phi_valid, double *rho_ave, int64_t *step) {
  if (!h) return LBPO_ERR_ARG;
  if (!h->initialised) return LBPO_ERR_STATE;
  if (f) memcpy(f, h->f, Q * h->n * sizeof(double));
  if (g) memcpy(g, h->g, Q * h->n * sizeof(double));
  if (phi_prev) memcpy(phi_prev, h->phi_prev, h->n * sizeof(double));
  if (phi_valid) *phi_valid = h->phi_valid;
  if (rho_ave) *rho_ave = h->rho_ave;
  if (step) *step = h->step;
  return LBPO_OK;
}

int lbpo_get_tv_prev(lbpo_handle *h, double *tv) {
  if (!h || !tv) return LBPO_ERR_ARG;
  memcpy(tv, h->tvx_prev, h->n * sizeof(double));
  memcpy(tv + h->n, h->tvy_prev, h->n * sizeof(double));
  return LBPO_OK;
}

int lbpo_set_tv_prev(lbpo_handle *h, const double *tv) {
  if (!h || !tv) return LBPO_ERR_ARG;
  memcpy(h->tvx_prev, tv, h->n * sizeof(double));
  memcpy(h->tvy_prev, tv + h->n, h->n * sizeof(double));
  return LBPO_OK;
}

int lbpo_set_state(lbpo_handle *h, const double *f, const double *g,
                   const double *phi_prev, int32_t phi_valid, double rho_ave,
                   int64_t step) {
  if (!h || !f || !g || !phi_prev) return LBPO_ERR_ARG;
  memcpy(h->f, f, Q * h->n * sizeof(double));
  memcpy(h->g, g, Q * h->n * sizeof(double));
  memcpy(h->phi_prev, phi_prev, h->n * sizeof(double));
  h->phi_valid = phi_valid ? 1 : 0;
  h->rho_ave = rho_ave;
  h->step = step;
  h->bad = 0;
  h->initialised = 1;
  return LBPO_OK;
}

void lbpo_iso_grad_lap(int nx, int ny, const double *X, double *dx, double *dy,
                       double *lap) {
  for (int y = 0; y < ny; ++y)
    for (int x = 0; x < nx; ++x) {
      size_t i = (size_t)y * nx + x;
      double sx = 0.0, sy = 0.0, sl = 0.0;
      for (int a = 1; a < Q; ++a) {
        int xx = (x + EX[a] + nx) % nx, yy = (y + EY[a] + ny) % ny;
        double Xn = X[(size_t)yy * nx + xx];
        sx += WL[a] * Xn * EX[a];
        sy += WL[a] * Xn * EY[a];
        sl += WL[a] * (Xn - X[i]);
      }
      dx[i] = sx / CS2;
      dy[i] = sy / CS2;
      lap[i] = sl * 2.0 / CS2;
    }
}
