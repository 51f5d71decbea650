/*
 * lbpo.h -- CPU ORACLE (test infrastructure only) for the coupled
 * pseudopotential-multiphase / improved-thermal MRT lattice Boltzmann step of
 * Li, Zhou & Yan, "Improved thermal lattice Boltzmann model for simulation of
 * liquid-vapor phase change" (arXiv:1709.04400).
 *
 * This is a plain, slow, single-threaded FP64 implementation written to be
 * read against the paper.  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load it.  It shares no source with the
 * GPU library; its configuration struct is declared here independently and a
 * test checks that the two layouts agree field by field.
 *
 * Lattice units throughout: dx = dt = c = 1, c_s^2 = 1/3.
 */
#ifndef LBPO_H
#define LBPO_H

#include <stdint.h>
#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbpo_handle lbpo_handle;

enum {
  LBPO_OK = 0,
  LBPO_ERR_ARG = -1,
  LBPO_ERR_OOM = -3,
  LBPO_ERR_STATE = -4,
  LBPO_ERR_NUMERIC = -5
};

/* boundary kinds, one per side (order x-, x+, y-, y+) */
enum { LBPO_BC_PERIODIC = 0, LBPO_BC_WALL = 1, LBPO_BC_OPEN = 2 };
/* thermal conductivity modes: constant, or lambda = rho c_V chi (Sec. IV) */
enum { LBPO_LAMBDA_CONST = 0, LBPO_LAMBDA_RHO_CV_CHI = 1 };
/* thermal models: the improved one of Sec. III.B; the "compromised" one of
 * Sec. IV that omits Eqs. (54)-(55) and the 0.5 dt d_t(phi) term of
 * Eq. (46); and the Gong-Cheng model of Sec. II.B, Eqs. (11)-(14): BGK
 * collision with the quadratic equilibrium of Eq. (14), source
 * G_a = omega_a phi with phi of Eq. (13), and the local relaxation time
 * tau_g = lambda / (rho c_V c_s^2) + 1/2 that makes chi = lambda/(rho c_V)
 * = (tau_g - 1/2) c_s^2 (Sec. II.B, below Eq. (25)) */
enum {
  LBPO_THERMAL_IMPROVED = 0,
  LBPO_THERMAL_COMPROMISED = 1,
  LBPO_THERMAL_GONG_CHENG = 2,
  /* the BGK form of the improved model, Sec. III.A, Eq. (33): equilibrium
   * of Eq. (29), correction C_a of Eq. (31), source of Eq. (32) with phi of
   * Eq. (28); one relaxation time tau_g = 1/s_g[3], so k = (tau_g - 1/2)
   * c_s^2 as in Eq. (41) */
  LBPO_THERMAL_IMPROVED_BGK = 3
};
/* test-only flags: flow field frozen (f never changes, F = 0); temperature
 * field frozen (g never changes) */
enum { LBPO_FLAG_FREEZE_FLOW = 1, LBPO_FLAG_FREEZE_THERMAL = 2 };

typedef struct lbpo_config {
  /* Peng-Robinson EOS, Eq. (56) */
  double a, b, R, omega;
  double cv;            /* specific heat at constant volume */
  double lambda0;       /* constant conductivity (LAMBDA_CONST) */
  double chi;           /* diffusivity when lambda = rho c_V chi */
  double s_f[9];        /* flow MRT relaxation rates */
  double s_g[9];        /* thermal MRT relaxation rates, Eq. (43) */
  double G;             /* pseudopotential interaction strength (< 0) */
  double sigma;         /* mechanical-stability constant of the flow forcing */
  double gx, gy;        /* gravity; buoyancy F_b = (rho - rho_ave) g */
  double T_bc[4];       /* wall / open temperatures, sides x-, x+, y-, y+ */
  double T_hot;         /* hot-spot temperature on the y- wall */
  double rho_ref, T_ref;/* shifted-storage references (GPU only; ignored) */
  double rho_v, rho_l;  /* coexistence densities used by the radius diagnostic */
  /* wetting of wall sides (a reading: the paper names contact angles but no
   * scheme): the interaction force sees a ghost node across a wall through
   * psi(rho_w, T_n) with the virtual density rho_w = (1 + wet_amp) rho_n -
   * wet_shift, clamped to [0, 0.9/b], of the ghost's nearest lattice node n
   * (rho_n, T_n).  Zero for both is the neutral rule psi = psi_n; wet_amp > 0
   * makes the wall more wetting, wet_shift > 0 less. */
  double wet_amp, wet_shift;
  int32_t nx, ny;
  int32_t bc[4];
  int32_t hot_x0, hot_x1;   /* hot spot covers hot_x0 <= x < hot_x1 */
  int32_t lambda_mode;
  int32_t thermal_model;
  int32_t precision;        /* GPU only; the oracle is always FP64 */
  uint32_t flags;
} lbpo_config;

typedef struct lbpo_diag {
  double mass;        /* sum rho */
  double sum_T;       /* sum T */
  double sum_rhocvT;  /* sum rho c_V T */
  double liquid_area; /* sum clamp((rho-rho_v)/(rho_l-rho_v), 0, 1) */
  double radius;      /* sqrt(liquid_area / pi) */
  double radius_count;/* sqrt(#{rho > (rho_l+rho_v)/2} / pi) */
  double max_speed;   /* max |v| */
  double sum_S0;      /* sum of the thermal source S0 of the last step */
  double sum_Fx, sum_Fy; /* sum of the total force of the last step */
  int64_t step;
  int32_t nonfinite;  /* 1 if a non-finite or invalid state was seen */
  int32_t pad;
} lbpo_diag;

/* field ids for lbpo_get_field (values at the current time level t) */
enum {
  LBPO_FIELD_RHO = 0, LBPO_FIELD_T, LBPO_FIELD_UX, LBPO_FIELD_UY,
  LBPO_FIELD_PSI, LBPO_FIELD_FX, LBPO_FIELD_FY, LBPO_FIELD_PHI_PREV,
  LBPO_FIELD_JX, LBPO_FIELD_JY
};

int lbpo_create(const lbpo_config *cfg, lbpo_handle **out);
void lbpo_destroy(lbpo_handle *h);
/* host arrays [ny][nx] row-major; f(0)=f^eq(rho,u), g(0)=g^eq(T,u) */
int lbpo_init_fields(lbpo_handle *h, const double *rho, const double *ux,
                     const double *uy, const double *T);
int lbpo_step(lbpo_handle *h, int64_t n);
int lbpo_get_rho_u_T(lbpo_handle *h, double *rho, double *ux, double *uy,
                     double *T);
int lbpo_get_field(lbpo_handle *h, int field, double *out);
int lbpo_get_diag(lbpo_handle *h, lbpo_diag *out);
/* canonical state: f(t) [9][ny][nx], g(t) [9][ny][nx], phi(t-1) [ny][nx] */
int lbpo_get_state(lbpo_handle *h, double *f, double *g, double *phi_prev,
                   int32_t *phi_valid, double *rho_ave, int64_t *step);
/* history T v(t - dt) of the BGK improved model, [2][ny][nx] (x then y);
 * zeros for the other models */
int lbpo_get_tv_prev(lbpo_handle *h, double *tv);
int lbpo_set_tv_prev(lbpo_handle *h, const double *tv);
int lbpo_set_state(lbpo_handle *h, const double *f, const double *g,
                   const double *phi_prev, int32_t phi_valid, double rho_ave,
                   int64_t step);

/* building blocks exposed for the pin tests */
void lbpo_matrix_M(double out[81]);
void lbpo_matrix_Minv(double out[81]);
void lbpo_flow_meq(double rho, double vx, double vy, double out[9]);
void lbpo_thermal_meq(double T, double vx, double vy, double out[9]);
/* D2Q9 equilibrium of the Gong-Cheng model, Eq. (14), per direction */
void lbpo_gc_geq(double T, double vx, double vy, double out[9]);
/* equilibrium linear in v, Eq. (29), per direction */
void lbpo_lin_geq(double T, double vx, double vy, double out[9]);
double lbpo_Tc(double a, double b, double R);
double lbpo_p_eos(const lbpo_config *cfg, double rho, double T);
double lbpo_dpdT(const lbpo_config *cfg, double rho, double T);
/* isotropic gradient / Laplacian of a periodic [ny][nx] field */
void lbpo_iso_grad_lap(int nx, int ny, const double *X, double *dx, double *dy,
                       double *lap);

#ifdef __cplusplus
}
#endif
#endif
