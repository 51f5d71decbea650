/*
 * lbpc.h -- C ABI of the MI355X (gfx950) library for the coupled
 * pseudopotential-multiphase / improved-thermal MRT lattice Boltzmann time
 * step of Li, Zhou & Yan, "Improved thermal lattice Boltzmann model for
 * simulation of liquid-vapor phase change" (arXiv:1709.04400).
 *
 * What one step computes, on every node of an nx x ny D2Q9 lattice (lattice
 * units, dx = dt = c = 1, c_s^2 = 1/3):
 *   - density rho, momentum j and temperature T = sum_a g_a (Sec. III.A);
 *   - the Peng-Robinson p_EOS(rho, T) of Eq. (56) and the pseudopotential
 *     psi = sqrt(2 (p_EOS - rho c_s^2) / G), its cancelling differences
 *     always in FP64;
 *   - the interaction force -G psi(x) sum_a w_a psi(x + e_a) e_a plus the
 *     buoyancy (rho - rho_ave) g of Sec. IV.B; v = (j + F/2) / rho;
 *   - the flow MRT collision with the pseudopotential forcing scheme the
 *     paper adopts for the flow field (Sec. III.B, cited there);
 *   - the thermal source phi of Eq. (28) (its underlined terms) from
 *     isotropic differences, S0 = phi + (phi - phi_prev)/2 (Eq. 46 with the
 *     backward difference of Sec. III.B);
 *   - the improved thermal MRT collision: Eqs. (45), (46), (53), (54), (55);
 *   - streaming, Eq. (47), with periodic, wall (halfway bounce-back and
 *     anti-bounce-back Dirichlet T, optional hot spot) or open (zero-gradient
 *     flow, fixed T) sides.
 *
 * Ownership: the caller owns every host array and the device workspace
 * (sized by lbpc_workspace_bytes, at least 256-byte aligned, alive until
 * lbpc_destroy returns).  The library owns the handle.  No call aborts;
 * every call returns an lbpc_status, and lbpc_last_error gives a message.
 * Calls on one handle are not thread-safe; different handles are
 * independent.  Device work is enqueued on the stream given at creation.
 * A handle (or batch) belongs to one device, the one holding its workspace
 * and stream: make it the current device (hipSetDevice) for every call on
 * it, creation included (the tile defaults, events and the host-mapped state
 * flag are taken on the current device).
 *
 * Environment, read when a handle or batch is created (scheduling only:
 * results never depend on it):
 *   LBPC_TILE_BW, LBPC_TILE_H      initial block width and rows per tile
 *   LBPC_TILE_HE                   with LBPC_TILE_H, FP64 and FP16 forms
 *                                  only: rows per tile of the two strips
 *                                  holding non-periodic x sides
 *   LBPC_XCD_ORDER=0               plain tile order instead of the
 *                                  XCD-aware one
 *   LBPC_GRAPH=1, LBPC_BATCH_GRAPH=1   replay steady steps from a captured
 *                                  hipGraph (needs a non-NULL stream)
 *   LBPC_PERSISTENT=1              tile-list kernel with one block per
 *                                  resident slot walking the list
 *   LBPC_FORCE_TILED=1, LBPC_FORCE_GEN=1   run a periodic lattice through
 *                                  the tile-list / boundary-capable kernel
 *   LBPC_TWO_STEP=1                two time steps per launch where
 *                                  available (lbpc_steps_per_launch)
 *   LBPC_STAGE_NODES=n             nodes per field of the FP64 staging
 *                                  scratch that initial fields, readback and
 *                                  checkpoints pass through in chunks
 *                                  (default 2^20, never under three rows);
 *                                  read by lbpc_workspace_bytes as well, so
 *                                  keep it fixed between that call and
 *                                  lbpc_create
 */
#ifndef LBPC_H
#define LBPC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lbpc_handle lbpc_handle;

typedef enum {
  LBPC_OK = 0,
  LBPC_ERR_ARG = -1,         /* invalid argument or configuration */
  LBPC_ERR_HIP = -2,         /* a HIP runtime call failed */
  LBPC_ERR_OOM = -3,         /* workspace too small / host allocation */
  LBPC_ERR_STATE = -4,       /* call out of order (e.g. step before init) */
  LBPC_ERR_NUMERIC = -5,     /* non-finite or invalid state detected */
  LBPC_ERR_UNSUPPORTED = -6  /* option not available on this path */
} lbpc_status;

/* storage precision of the distributions (arithmetic: FP64 for FP64, FP32
 * otherwise, whose reciprocals and square roots are the hardware's, within
 * 1 ulp; the EOS's cancelling differences, repulsive minus attractive
 * pressure and p - rho c_s^2, and the diagnostic sums are always FP64).  The
 * shifted forms store f_a - w_a rho_ref and g_a - wg_a T_ref, with w the
 * D2Q9 weights and wg = (5/9, 1/18, ..., 1/18) the rest equilibrium of
 * Eq. (53).  Below FP64, f and g of a direction are stored as one (f, g)
 * pair (8 bytes in FP32).  LBPC_FP16_SHIFTED keeps the deviations of
 * directions 1-8 as binary16, the pair in one 32-bit word, and the rest
 * populations as an FP32 pair per node, each less the rounding errors of
 * its node's other eight.  LBPC_FP16_LOCAL stores the same words against
 * node-local references instead of rho_ref and T_ref: each node keeps a
 * binary16 (rho, T) of its own in its direction-0 word, and the value a
 * node sends in direction a is stored less w_a rho and wg_a T of the node
 * that will pull it (x + e_a; itself across a wall), so binary16 holds only
 * the velocity and non-equilibrium parts; the rest populations are FP32
 * full values (96 bytes moved per node and step against 88).  The
 * reference fields of lbpc_config are not used by it. */
typedef enum {
  LBPC_FP64 = 0,
  LBPC_FP32 = 1,
  LBPC_FP32_SHIFTED = 2,
  LBPC_FP16_SHIFTED = 3,
  LBPC_FP16_LOCAL = 4
} lbpc_precision;

/* side kinds; sides are ordered x-, x+, y-, y+.  Opposite sides are both
 * periodic or both not. */
typedef enum {
  LBPC_BC_PERIODIC = 0,
  LBPC_BC_WALL = 1, /* no-slip halfway bounce-back; T fixed (anti-bounce-back) */
  LBPC_BC_OPEN = 2  /* zero-gradient flow; incoming g at rest equilibrium T */
} lbpc_bc;

typedef enum { LBPC_LAMBDA_CONST = 0, LBPC_LAMBDA_RHO_CV_CHI = 1 } lbpc_lambda;
/* The improved model of Sec. III.B; the "compromised" one of Sec. IV without
 * Eqs. (54)-(55) and without the (phi - phi_prev)/2 term */
typedef enum {
  LBPC_THERMAL_IMPROVED = 0,
  LBPC_THERMAL_COMPROMISED = 1,
  /* the Gong-Cheng model of Sec. II.B, Eqs. (11)-(14): BGK collision with the
   * quadratic equilibrium of Eq. (14), source omega_a phi with phi of
   * Eq. (13), and the local relaxation time tau_g = lambda/(rho c_V c_s^2)
   * + 1/2; s_g is not used.  Its side rules use the rest weights omega_a of
   * Eq. (14) in place of those of Eq. (53).  Needs lambda0 > 0 (constant
   * conductivity) or chi > 0 (lambda = rho c_V chi). */
  LBPC_THERMAL_GONG_CHENG = 2,
  /* the BGK form of the improved model, Sec. III.A, Eq. (33): BGK relaxation
   * with tau_g = 1/s_g[3] towards the equilibrium of Eq. (29), the source
   * omega_a (phi + (phi - phi_prev)/2) of Eq. (32) with phi of Eq. (28), and
   * the correction of Eq. (31) with d_t(T v) taken as the backward
   * difference T v(t) - T v(t - 1) (zero on the first step).  It keeps T v
   * of the previous step per node, which adds 2 values per node to the
   * workspace and to the saved state.  Side rules use the rest weights
   * omega_a of Eq. (29). */
  LBPC_THERMAL_IMPROVED_BGK = 3
} lbpc_thermal_model;

/* Ghost rule at a non-periodic side, used by every stencil: a neighbour
 * outside the lattice takes rho and psi of the nearest lattice node (psi
 * from the virtual density of wet_amp / wet_shift across a wall), v = 0
 * at a wall (v of that node at an open side) and T of the crossed side (y
 * side first at corners; the y- wall has T_hot on hot_x0 <= x < hot_x1).
 *
 * Field order and types match the oracle's configuration struct exactly
 * (a test compares the two layouts). */
typedef struct lbpc_config {
  double a, b, R, omega;  /* Peng-Robinson EOS, Eq. (56) */
  double cv;              /* specific heat at constant volume */
  double lambda0;         /* conductivity for LBPC_LAMBDA_CONST */
  double chi;             /* lambda = rho c_V chi for LBPC_LAMBDA_RHO_CV_CHI */
  double s_f[9];          /* flow MRT rates, moments (rho,e,eps,jx,qx,jy,qy,pxx,pxy) */
  double s_g[9];          /* thermal MRT rates, Eq. (43); k = (1/s_g[3]-1/2)/3 */
  double G;               /* interaction strength, < 0 */
  double sigma;           /* forcing-scheme constant (flow model) */
  double gx, gy;          /* gravity for the buoyancy (rho - rho_ave) g */
  double T_bc[4];         /* side temperatures (wall / open sides) */
  double T_hot;           /* hot-spot temperature on the y- wall */
  double rho_ref, T_ref;  /* references of the shifted storage forms */
  double rho_v, rho_l;    /* coexistence densities for the radius diagnostic */
  double wet_amp;         /* wall wetting: a ghost across a wall enters the */
  double wet_shift;       /* interaction force with psi(rho_w, T_n), rho_w =
                           * (1 + wet_amp) rho_n - wet_shift clamped to
                           * [0, 0.9/b], n the nearest lattice node; 0 and 0
                           * give psi_n (neutral); wet_amp > -1, finite */
  int32_t nx, ny;         /* lattice size, each >= 4 */
  int32_t bc[4];          /* lbpc_bc per side */
  int32_t hot_x0, hot_x1; /* hot-spot columns */
  int32_t lambda_mode;    /* lbpc_lambda */
  int32_t thermal_model;  /* lbpc_thermal_model */
  int32_t precision;      /* lbpc_precision */
  uint32_t flags;         /* must be 0 (the oracle's test-only flags) */
} lbpc_config;

/* FP64 sums over the lattice at one time level (the paper reports the
 * droplet diameter ratio D/D0 of Sec. IV.A but defines no measure; these
 * are the readings the library uses).  rho, T and v are the fields of the
 * step's own arithmetic at that level (FP32 in the reduced-precision forms),
 * summed in FP64. */
typedef struct lbpc_diag {
  double mass;         /* sum rho */
  double sum_T;        /* sum T */
  double sum_rhocvT;   /* sum rho c_V T */
  double liquid_area;  /* sum clamp((rho - rho_v)/(rho_l - rho_v), 0, 1) */
  double radius;       /* sqrt(liquid_area / pi) */
  double radius_count; /* sqrt(#{rho > (rho_l + rho_v)/2} / pi) */
  double max_speed;    /* max |v| */
  double sum_S0;       /* sum of the thermal source S0 of Eq. (46) of the
                        * step taken from this level (sum T of the next
                        * level is sum T + sum S0 on periodic lattices) */
  int64_t step;        /* the time level: steps since lbpc_init_fields */
  int32_t nonfinite;   /* 1 if a non-finite value or an invalid state
                        * (flagged by a step) was seen */
  int32_t pad;
} lbpc_diag;

/* Device bytes the caller must provide for this configuration: two
 * population buffers (FP64: f and g, nine nx*ny arrays apiece; below FP64
 * nine arrays of (f, g) pairs, and in the FP16 deviation form an FP32 rest
 * pair per node), two copies of the phi history, a staging scratch of at
 * most 40 MiB by default (five FP64 fields of LBPC_STAGE_NODES nodes) and
 * the tile list with its diagnostic records. */
lbpc_status lbpc_workspace_bytes(const lbpc_config *cfg, size_t *bytes);

/* Validates cfg and binds the workspace and stream (hipStream_t, may be
 * NULL for the null stream).  Nothing is launched; besides the handle the
 * library allocates one 4-byte pinned host flag (host-mapped), which the
 * step kernel sets on an invalid node state.  On failure *out is NULL. */
lbpc_status lbpc_create(const lbpc_config *cfg, void *dev_workspace,
                        size_t workspace_bytes, void *hip_stream,
                        lbpc_handle **out);

/* Initial fields: host FP64 arrays, row-major [ny][nx], copied (the call
 * returns after the copy).  Sets f = f^eq(rho, u), g = g^eq(T, u) (the
 * equilibrium of the thermal model: Eq. 53 moments mapped back by M^-1, or
 * Eq. 14 / Eq. 29 for the BGK models), rho_ave = mean rho, step = 0, marks
 * phi_prev as unset (the first step uses phi_prev = phi) and clears the
 * invalid-state flag.  Rejects rho <= 0, rho >= 1/b, T <= 0, a negative
 * psi^2 or non-finite values (LBPC_ERR_ARG). */
lbpc_status lbpc_init_fields(lbpc_handle *h, const double *rho,
                             const double *ux, const double *uy,
                             const double *T);

/* Enqueues n >= 0 coupled time steps on the stream and returns without
 * waiting.  With LBPC_GRAPH=1 in the environment at lbpc_create and a
 * non-NULL stream, steady-state pairs of steps are replayed from a captured
 * hipGraph of one ping-pong period (same results; on MI355X eager launches
 * measured slightly faster, so it is off by default).  Each step checks
 * every node's state (psi^2 >= 0, 0 < rho < 1/b, finite T: the conditions
 * under which psi of Eq. (56) and the collision are defined) and flags a
 * violation.
 * A flag set by a step that has completed makes lbpc_step return
 * LBPC_ERR_NUMERIC without enqueuing; every synchronising call
 * (lbpc_get_rho_u_T, lbpc_get_diag, lbpc_save_state) reports it exactly.
 * lbpc_load_state (of a good state) and lbpc_init_fields clear it. */
lbpc_status lbpc_step(lbpc_handle *h, int64_t n);

/* Tile shape of the step launches: threads per block (64, 128, 256 or 512;
 * the strip is at most that many columns minus 4 halo columns) and rows per
 * tile (>= 4), the same for every strip.  Results do not depend on it.
 * Default: 512 for FP64 and for the periodic FP32 forms, 256 otherwise;
 * rows: the height that makes the tile count just fill a whole number of
 * waves of resident blocks (for the FP32 forms on a lattice with a
 * non-periodic side: three waves). */
lbpc_status lbpc_set_tiles(lbpc_handle *h, int32_t block_width, int32_t rows);

/* The tile shape in place: threads per block, rows per tile, and rows per
 * tile of the two strips that hold the x sides when those are not periodic,
 * in FP64 and the FP16 forms (equal to rows otherwise, and after
 * lbpc_set_tiles).  Any output pointer
 * may be NULL; LBPC_ERR_ARG if h is NULL.  Host only: no device work. */
lbpc_status lbpc_get_tiles(const lbpc_handle *h, int32_t *block_width,
                           int32_t *rows, int32_t *rows_edge);

/* Time steps per launch of lbpc_step: 2 where it runs two steps in one
 * launch (on request, LBPC_TWO_STEP=1 at creation: the FP32 and
 * FP32-deviation forms on periodic lattices of at least 16 x 16 nodes under
 * the improved or compromised model, without graph replay; the results
 * agree with single steps to FP32 rounding; an odd last step runs alone),
 * else 1.
 * The two-step launches keep their own tile shape (256-thread blocks, one
 * block per CU); lbpc_set_tiles and lbpc_autotune set the single-step
 * shape.  Host only. */
lbpc_status lbpc_steps_per_launch(const lbpc_handle *h, int32_t *steps);

/* Times `steps` launches of each candidate tile shape (the shape in place;
 * block width 64, 128, 256, 512 x rows 4 ... 64 and that width's default
 * rows) on the current state, keeps the fastest and reports it.  State and phi history are left unchanged (timing launches write phi
 * to scratch).  Blocks until done. */
lbpc_status lbpc_autotune(lbpc_handle *h, int32_t steps, int32_t *block_width,
                          int32_t *rows, double *ms_per_step);

/* Measurement aid: times `launches` launches of the step kernel's memory
 * schedule with its arithmetic left out (every node stores the values it
 * pulls and its phi history: the same loads and stores, tile shape and
 * march order as lbpc_step) on the current state, which it leaves as it is,
 * and reports the mean milliseconds per launch.  The step moves the same
 * bytes per launch, so its time over this one is the share of the bandwidth
 * its access pattern can reach that it attains.  Periodic lattices on
 * 256- or 512-thread tiles only (LBPC_ERR_UNSUPPORTED otherwise).  Blocks
 * until done. */
lbpc_status lbpc_memory_probe(lbpc_handle *h, int32_t launches,
                              double *ms_per_launch);

/* Waits for the stream; writes rho, v = (j + F/2)/rho and T at the current
 * time level into host FP64 arrays [ny][nx] (any pointer may be NULL).
 * Returns LBPC_ERR_NUMERIC if a non-finite value is present. */
lbpc_status lbpc_get_rho_u_T(lbpc_handle *h, double *rho, double *ux,
                             double *uy, double *T);

/* Diagnostics of the current time level without stepping: one pass of the
 * fused step kernel that computes the level's fields and S0 and reduces
 * them (waves, then blocks, then a fixed-order final pass: the same result
 * on every run) but stores nothing, so the state is left as it is.  Waits
 * for it and fills *out; returns LBPC_ERR_NUMERIC (with *out filled and
 * nonfinite = 1) when a step has flagged an invalid state or a value is
 * not finite. */
lbpc_status lbpc_get_diag(lbpc_handle *h, lbpc_diag *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation):
 * lbpc_get_diag with its tile records and results in a static device array
 * of the library instead of the workspace.  The array holds 65536 tile
 * records (4 MiB with the results); every GPU the library runs on keeps its
 * own copy until the process ends.  The call allocates nothing and sets no
 * memory; it returns LBPC_ERR_UNSUPPORTED when the handle's tile shape has
 * more than 65536 tiles (use taller tiles, or lbpc_get_diag).  Every call on
 * one GPU uses that GPU's array, so calls that overlap on one GPU (several
 * threads, or several streams in flight) race; each call waits for its
 * result before returning.  Same values as lbpc_get_diag (bitwise). */
lbpc_status lbpc_get_diag_noalloc(lbpc_handle *h, lbpc_diag *out);

/* Enqueues n >= 1 time steps like lbpc_step; the first of them also
 * reduces the diagnostics of the time level it starts from (the current
 * one), on the way, in the same launch.  Returns once that first step's
 * results are in *out (out->step is that level), while the other n - 1
 * steps may still run.  Same values as lbpc_get_diag called before the
 * steps.  Errors as lbpc_step and lbpc_get_diag. */
lbpc_status lbpc_step_diag(lbpc_handle *h, int64_t n, lbpc_diag *out);

/* Canonical state {f(t) [9][ny][nx], g(t) [9][ny][nx], phi(t-1) [ny][nx]}
 * as FP64 (for the BGK form of the improved model followed by T v_x and
 * T v_y of step t-1, [ny][nx] each), then phi_valid, rho_ave and step as
 * three 8-byte words: lbpc_state_bytes gives the host buffer size.  Save
 * waits for the stream and refuses (LBPC_ERR_NUMERIC) a flagged state.  A
 * loaded state resumes the run bit for bit, except in LBPC_FP16_LOCAL,
 * whose node references are not part of it: a load stores each value
 * against a reference taken from its node's rest populations (rho_ref =
 * f_0 / w_0, T_ref = g_0 / wg_0), which changes the first step's values by
 * their binary16 rounding. */
lbpc_status lbpc_state_bytes(const lbpc_handle *h, size_t *bytes);
lbpc_status lbpc_save_state(lbpc_handle *h, void *host, size_t bytes);
lbpc_status lbpc_load_state(lbpc_handle *h, const void *host, size_t bytes);

/* Waits for outstanding work, then frees the handle (NULL-safe).  The
 * workspace stays the caller's. */
void lbpc_destroy(lbpc_handle *h);

/* Message of the last failure on h (or of the calling thread's last failed
 * lbpc_create / lbpc_workspace_bytes when h is NULL).  Never NULL. */
const char *lbpc_last_error(const lbpc_handle *h);

/* ------------------------------------------------------------- batches --
 * Many independent lattices (different sizes, sides and parameters, one
 * storage precision) advanced together: one persistent kernel launch per
 * time step walks a list of (lattice, tile) work items, costliest first.
 * Every lattice computes exactly what a single handle with its
 * configuration computes.  With LBPC_BATCH_GRAPH=1 in the environment at
 * creation and a non-NULL stream, steady-state steps are replayed from a
 * captured hipGraph of two steps (one ping-pong period); off by default
 * (eager launches measured slightly faster). */
typedef struct lbpc_batch lbpc_batch;

/* Device bytes for the batch (all lattices, the work list, shared scratch). */
lbpc_status lbpc_batch_workspace_bytes(const lbpc_config *cfgs, int32_t n,
                                       size_t *bytes);
/* cfgs[0..n-1]: one configuration per lattice, same precision, flags 0. */
lbpc_status lbpc_batch_create(const lbpc_config *cfgs, int32_t n,
                              void *dev_workspace, size_t workspace_bytes,
                              void *hip_stream, lbpc_batch **out);
/* Initial fields of lattice c (host FP64 [ny][nx], copied; same rules as
 * lbpc_init_fields).  Allowed only before the first step; every lattice must
 * be initialised before lbpc_batch_step. */
lbpc_status lbpc_batch_init_fields(lbpc_batch *b, int32_t c,
                                   const double *rho, const double *ux,
                                   const double *uy, const double *T);
/* Tile shape: threads per block (64, 128, 256 or 512) and rows per tile
 * (>= 4). */
lbpc_status lbpc_batch_set_tiles(lbpc_batch *b, int32_t block_width,
                                 int32_t rows);
/* Times `steps` launches of each candidate tile shape (the shape in place;
 * block width 64, 128, 256 x rows 16, 20, 24, 32, 48, 64) on the current
 * state, keeps the fastest and reports it.  The state and the phi history are left unchanged (timing
 * launches write phi to scratch).  Before the first step the launches read
 * the initial state in place, so tune after a step for steady-state
 * timings.  Blocks until done. */
lbpc_status lbpc_batch_autotune(lbpc_batch *b, int32_t steps,
                                int32_t *block_width, int32_t *rows,
                                double *ms_per_step);
/* Enqueues n coupled time steps of every lattice. */
lbpc_status lbpc_batch_step(lbpc_batch *b, int64_t n);
/* Per-lattice readback, as lbpc_get_rho_u_T / lbpc_get_diag (synchronising;
 * the diagnostic pass covers every lattice of the batch). */
lbpc_status lbpc_batch_get_rho_u_T(lbpc_batch *b, int32_t c, double *rho,
                                   double *ux, double *uy, double *T);
lbpc_status lbpc_batch_get_diag(lbpc_batch *b, int32_t c, lbpc_diag *out);
/* As lbpc_step_diag for every lattice: n >= 1 steps, the first of which also
 * reduces each lattice's diagnostics of the current time level into
 * out[0 .. count-1] (count = the number of lattices). */
lbpc_status lbpc_batch_step_diag(lbpc_batch *b, int64_t n, lbpc_diag *out);
/* Lattice-node updates per step summed over the batch (for throughput). */
lbpc_status lbpc_batch_nodes(const lbpc_batch *b, int64_t *nodes);
void lbpc_batch_destroy(lbpc_batch *b);
const char *lbpc_batch_last_error(const lbpc_batch *b);

#ifdef __cplusplus
}
#endif
#endif /* LBPC_H */
