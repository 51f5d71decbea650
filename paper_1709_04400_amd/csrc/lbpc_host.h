// lbpc_host.h -- host-side pieces shared by the single-lattice and the
// batched runtimes: launcher declarations, configuration checks, the derived
// constants of a lattice and the Peng-Robinson checks of the inputs.
#pragma once
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/lbpc.h"
#include "lbpc_device.h"

namespace lbpc {
hipError_t launch_step(const StepParams& p, int prec, hipStream_t s,
                       double* dpart = nullptr, int nostore = 0);
hipError_t launch_step_probe(const StepParams& p, int prec, hipStream_t s);
hipError_t launch_two_steps(const StepParams& p, int prec, hipStream_t s);
hipError_t launch_init(const StepParams& p, int prec, const double* in,
                       long long i0, long long cnt, hipStream_t s);
hipError_t launch_macro(const StepParams& p, int prec, double* io, int y0,
                        int nr, hipStream_t s);
hipError_t launch_diag_reduce(const double* part, const int* ranges, int lo,
                              int hi, int nlat, double* out, hipStream_t s);
hipError_t launch_canon(const StepParams& p, int prec, int which, double* out,
                        long long i0, long long cnt, hipStream_t s);
hipError_t launch_load(const StepParams& p, int prec, int which,
                       const double* in, long long i0, long long cnt,
                       hipStream_t s);
hipError_t launch_phi_out(const StepParams& p, int prec, double* out,
                          long long i0, long long cnt, hipStream_t s);
hipError_t launch_phi_in(const StepParams& p, int prec, const double* in,
                         long long i0, long long cnt, hipStream_t s);
hipError_t launch_step_batch(const StepParams* table, const void* work,
                             int nwork, int parity, int grid, int prec,
                             int bw, hipStream_t s, bool gen = true,
                             double* dpart = nullptr, int nostore = 0);
int work_item_bytes();
}  // namespace lbpc

using lbpc::StepParams;

namespace lbpc_host {

constexpr size_t ALIGN = 256;
inline size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

// Bytes of the f (k = 0) or g (k = 1) populations of one buffer.  FP64:
// nine nx*ny arrays each.  The other forms keep f and g of a direction as
// one (f, g) pair (8 bytes in FP32, a 32-bit word in FP16), nine nx*ny
// arrays of pairs, all in the f array; their g pointer aliases it.
inline bool fp16_form(int prec) {
  return prec == LBPC_FP16_SHIFTED || prec == LBPC_FP16_LOCAL;
}
inline size_t dist_bytes(const lbpc_config& c, int k) {
  const size_t n9 = 9 * (size_t)c.nx * (size_t)c.ny;
  switch (c.precision) {
    case LBPC_FP64: return n9 * 8;
    case LBPC_FP16_SHIFTED:
    case LBPC_FP16_LOCAL: return k == 0 ? n9 * 4 : 0;
    default: return k == 0 ? n9 * 8 : 0;
  }
}
inline size_t compute_bytes(int prec) { return prec == LBPC_FP64 ? 8 : 4; }
// per-node history arrays (compute precision): phi(t-1), and for the BGK
// form of the improved model also T v_x and T v_y of the previous step
inline int hist_arrays(const lbpc_config& c) {
  return c.thermal_model == LBPC_THERMAL_IMPROVED_BGK ? 3 : 1;
}

// FP32 rest populations of the FP16 forms, per buffer: an (f_0, g_0) pair
// per node, [N][2] (none for the other forms)
inline size_t rest_bytes(const lbpc_config& c) {
  return fp16_form(c.precision)
             ? 2 * (size_t)c.nx * (size_t)c.ny * sizeof(float)
             : 0;
}

// Nodes per field of the FP64 staging scratch through which initial
// fields, field readback and checkpoints pass, in chunks of nodes or bands
// of rows: the whole lattice and its two halo rows when that is at most
// `cap` nodes, else `cap` nodes (never under three rows, the smallest
// band).  Five fields of it: with the default cap of 2^20 nodes, 40 MiB
// instead of 40 B per node.  LBPC_STAGE_NODES sets the cap when a handle is
// created (smaller caps exercise the chunked transfers on small lattices).
inline size_t stage_cap() {
  const char* v = std::getenv("LBPC_STAGE_NODES");
  const long long c = v ? std::atoll(v) : 0;
  return c > 0 ? (size_t)c : (size_t)1 << 20;
}
inline size_t stage_nodes(int nx, int ny, size_t cap) {
  const size_t whole = ((size_t)ny + 2) * (size_t)nx;
  return std::min(whole, std::max(cap, 3 * (size_t)nx));
}

struct Layout {
  size_t dist[2][2];  // offsets of f / g of buffer 0 / 1
  size_t rest[2];     // FP16 deviation form: rest populations of buffer 0 / 1
  size_t phi, scratch, partial, diag_out;
  size_t stage;        // nodes per field of the staging scratch
  size_t table, work;  // parameter table and tile list (non-periodic path)
  size_t work_capacity;
  size_t tune_phi;     // phi(t) of the autotuner's timing launches
  size_t total;
};

// Strips of a lattice row for blocks of bw threads: as few as the block
// width allows, either full (bw - 4 columns, the last strip taking the
// remainder) or balanced (all of about the same width).  Balanced strips
// spread a row run evenly over its blocks instead of leaving one narrow
// strip to a nearly idle block; measured at 4096^2 they speed up the FP64
// step (+1.6 %) and mixed-size batches (+1 %) but slow the single-lattice
// FP32 forms (-2 to -4.5 %), which therefore keep full strips.
// Single lattices: balanced strips for FP64, and for any form with 512-thread
// blocks, where a full split leaves a nearly empty last strip (4096 columns:
// 8 x 508 + 32); FP32 at 512 ran +1.4 % balanced, FP32 deviations +0.7 %.
inline bool balanced_strips(int precision, int bw) {
  return precision == LBPC_FP64 || bw == 512;
}

inline void strip_shape(int nx, int bw, bool balanced, int& nbx, int& W) {
  const int wmax = bw - 2 * lbpc::HALO;
  nbx = (nx + wmax - 1) / wmax;
  W = balanced ? (nx + nbx - 1) / nbx : wmax;
}

inline Layout plan(const lbpc_config& c) {
  Layout L;
  const size_t N = (size_t)c.nx * (size_t)c.ny;
  size_t off = 0;
  for (int b = 0; b < 2; ++b) {
    for (int k = 0; k < 2; ++k) {
      L.dist[b][k] = off;
      off += align_up(dist_bytes(c, k));
    }
    if (dist_bytes(c, 1) == 0) L.dist[b][1] = L.dist[b][0];
  }
  for (int b = 0; b < 2; ++b) {
    L.rest[b] = off;
    off += align_up(rest_bytes(c));
  }
  const size_t hbytes = align_up(hist_arrays(c) * N * compute_bytes(c.precision));
  L.phi = off;
  off += hbytes;
  L.stage = stage_nodes(c.nx, c.ny, stage_cap());
  L.scratch = off;
  off += align_up(5 * L.stage * sizeof(double));
  // tiles of the narrowest strips (60 columns) and shortest runs (4 rows):
  // the most any tile shape makes, each with one diagnostic record
  L.work_capacity = (size_t)((c.nx + 59) / 60) * (size_t)((c.ny + 3) / 4);
  L.partial = off;
  off += align_up(L.work_capacity * 8 * sizeof(double));
  L.diag_out = off;
  off += align_up(8 * sizeof(double));
  L.table = off;
  off += align_up(2 * sizeof(StepParams));
  L.work = off;
  off += align_up(L.work_capacity * 16);
  L.tune_phi = off;
  off += hbytes;
  L.total = off;
  return L;
}

inline double pr_Tc(const lbpc_config& c) {
  return 0.0778 * c.a / (0.45724 * c.b * c.R);
}
inline double pr_kappa(double w) { return 0.37464 + 1.54226 * w - 0.26992 * w * w; }

inline double host_psi2(const lbpc_config& c, double rho, double T) {
  const double Tc = pr_Tc(c), k = pr_kappa(c.omega);
  const double s = 1.0 + k * (1.0 - std::sqrt(T / Tc));
  const double p = rho * c.R * T / (1.0 - c.b * rho) -
                   c.a * s * s * rho * rho /
                       (1.0 + 2.0 * c.b * rho - c.b * c.b * rho * rho);
  return 2.0 * (p - rho * (1.0 / 3.0)) / c.G;
}

inline const char* check_config(const lbpc_config* c) {
  if (!c) return "config is NULL";
  if (c->nx < 4 || c->ny < 4) return "nx and ny must be >= 4";
  if ((long long)c->nx * (long long)c->ny > (1LL << 31))
    return "lattice larger than 2^31 nodes";
  for (int i = 0; i < 4; ++i)
    if (c->bc[i] < 0 || c->bc[i] > 2) return "bc must be 0, 1 or 2";
  if ((c->bc[0] == LBPC_BC_PERIODIC) != (c->bc[1] == LBPC_BC_PERIODIC))
    return "x sides must be both periodic or both not";
  if ((c->bc[2] == LBPC_BC_PERIODIC) != (c->bc[3] == LBPC_BC_PERIODIC))
    return "y sides must be both periodic or both not";
  for (int i = 0; i < 9; ++i)
    if (!(c->s_f[i] > 0.0 && c->s_f[i] < 2.0) ||
        !(c->s_g[i] > 0.0 && c->s_g[i] < 2.0))
      return "relaxation rates must lie in (0, 2)";
  if (!(c->G < 0.0)) return "G must be negative";
  if (!std::isfinite(c->wet_amp) || !(c->wet_amp > -1.0) ||
      !std::isfinite(c->wet_shift))
    return "wet_amp must be finite and > -1, wet_shift finite";
  if (!(c->a > 0.0 && c->b > 0.0 && c->R > 0.0 && c->cv > 0.0))
    return "a, b, R and cv must be positive";
  if (c->lambda_mode != LBPC_LAMBDA_CONST &&
      c->lambda_mode != LBPC_LAMBDA_RHO_CV_CHI)
    return "unknown lambda_mode";
  if (c->thermal_model != LBPC_THERMAL_IMPROVED &&
      c->thermal_model != LBPC_THERMAL_COMPROMISED &&
      c->thermal_model != LBPC_THERMAL_GONG_CHENG &&
      c->thermal_model != LBPC_THERMAL_IMPROVED_BGK)
    return "unknown thermal_model";
  if (c->thermal_model == LBPC_THERMAL_GONG_CHENG &&
      !(c->lambda_mode == LBPC_LAMBDA_CONST ? c->lambda0 > 0.0 : c->chi > 0.0))
    return "the Gong-Cheng model needs lambda0 > 0 or chi > 0";
  if (c->precision < LBPC_FP64 || c->precision > LBPC_FP16_LOCAL)
    return "unknown precision";
  return nullptr;
}

// Per-lattice constants of the step kernels (buffers, state flags and the
// tile shape are filled in by the caller).
inline void derive_params(const lbpc_config& c, StepParams& p) {
  std::memset(&p, 0, sizeof(p));
  p.nx = c.nx;
  p.ny = c.ny;
  p.perx = c.bc[0] == LBPC_BC_PERIODIC;
  p.pery = c.bc[2] == LBPC_BC_PERIODIC;
  for (int i = 0; i < 4; ++i) {
    p.bc[i] = c.bc[i];
    p.T_bc[i] = c.T_bc[i];
  }
  p.hot_x0 = c.hot_x0;
  p.hot_x1 = c.hot_x1;
  p.T_hot = c.T_hot;
  p.a = c.a;
  p.b = c.b;
  p.R = c.R;
  p.Tc = pr_Tc(c);
  p.kappa = pr_kappa(c.omega);
  p.G = c.G;
  p.sigma = c.sigma;
  p.gx = c.gx;
  p.gy = c.gy;
  for (int i = 0; i < 9; ++i) {
    p.s_f[i] = c.s_f[i];
    p.s_g[i] = c.s_g[i];
  }
  p.cv = c.cv;
  p.lambda0 = c.lambda0;
  p.chi = c.chi;
  p.k_th = (1.0 / c.s_g[3] - 0.5) * (1.0 / 3.0);  // Eq. (A13), c_s^2 = 1/3
  p.inv_Tc = 1.0 / p.Tc;
  p.two_over_G = 2.0 / c.G;
  p.inv_cv = 1.0 / c.cv;
  p.lam_over_cv = c.lambda0 / c.cv;
  p.sig1 = 12.0 * c.sigma * c.G * c.G / (1.0 / c.s_f[1] - 0.5);
  p.sig2 = 12.0 * c.sigma * c.G * c.G / (1.0 / c.s_f[2] - 0.5);
  p.lambda_mode = c.lambda_mode;
  p.improved = c.thermal_model == LBPC_THERMAL_IMPROVED;
  p.gc = c.thermal_model == LBPC_THERMAL_GONG_CHENG;
  p.bgk = c.thermal_model == LBPC_THERMAL_IMPROVED_BGK;
  p.wet = c.wet_amp != 0.0 || c.wet_shift != 0.0;
  p.wet_amp = c.wet_amp;
  p.wet_shift = c.wet_shift;
  // BGK form: 1/tau_g = s_g[3]; (1 - 1/(2 tau_g)) / c_s^2 of Eq. (31)
  p.bgk_itau = c.s_g[3];
  p.bgk_cfac = 3.0 * (1.0 - 0.5 * c.s_g[3]);
  if (p.gc || p.bgk) {
    // rest equilibrium of Eqs. (14) and (29): the D2Q9 weights
    p.wg0 = 4.0 / 9.0;
    p.wg1 = 1.0 / 9.0;
    p.wg2 = 1.0 / 36.0;
    // tau_g = lambda / (rho c_V c_s^2) + 1/2 = gc_ta / rho + gc_tb
    if (!p.gc) {
      p.gc_ta = 0.0;
      p.gc_tb = 0.0;
    } else if (c.lambda_mode == LBPC_LAMBDA_CONST) {
      p.gc_ta = 3.0 * c.lambda0 / c.cv;
      p.gc_tb = 0.5;
    } else {
      p.gc_ta = 0.0;
      p.gc_tb = 3.0 * c.chi + 0.5;
    }
  } else {
    // rest equilibrium of Eq. (53): M^-1 (1, -2, 2, 0, ..., 0)
    p.wg0 = 5.0 / 9.0;
    p.wg1 = 1.0 / 18.0;
    p.wg2 = 1.0 / 18.0;
  }
  p.rho_ref = c.rho_ref;
  p.T_ref = c.T_ref;
  p.rho_v = c.rho_v;
  p.rho_l = c.rho_l;
  p.N = (long long)c.nx * c.ny;
}

// Host checks of initial fields (same rules as the library documents):
// returns nullptr when valid, and the mean density in *rho_ave.
inline const char* check_fields(const lbpc_config& c, const double* rho,
                                const double* ux, const double* uy,
                                const double* T, double* rho_ave) {
  const size_t N = (size_t)c.nx * c.ny;
  double sum = 0.0;
  for (size_t i = 0; i < N; ++i) {
    if (!(rho[i] > 0.0 && rho[i] < 1.0 / c.b)) return "rho outside (0, 1/b)";
    if (!(T[i] > 0.0) || !std::isfinite(T[i]) || !std::isfinite(ux[i]) ||
        !std::isfinite(uy[i]))
      return "T <= 0 or non-finite input";
    if (!(host_psi2(c, rho[i], T[i]) >= 0.0))
      return "psi^2 < 0 (p_EOS > rho c_s^2)";
    sum += rho[i];
  }
  *rho_ave = sum / (double)N;
  return nullptr;
}

// Fills a diagnostic record from the 8 reduced values (sum rho, sum T,
// sum rho T, liquid area, count, sum S0, max |v|^2, non-finite) of the time
// level `step`.
inline void fill_diag(lbpc_diag* out, const double* r, double cv,
                      int64_t step, bool flagged) {
  std::memset(out, 0, sizeof(*out));
  out->mass = r[0];
  out->sum_T = r[1];
  out->sum_rhocvT = cv * r[2];
  out->liquid_area = r[3];
  out->radius = std::sqrt(r[3] / M_PI);
  out->radius_count = std::sqrt(r[4] / M_PI);
  out->sum_S0 = r[5];
  out->max_speed = std::sqrt(r[6]);
  out->step = step;
  out->nonfinite = (r[7] != 0.0 || !std::isfinite(r[0]) ||
                    !std::isfinite(r[1]) || !std::isfinite(r[5]) || flagged)
                       ? 1
                       : 0;
}

// Order tiles for the XCDs: workgroup w runs on XCD w % 8, so item w gets
// tile t of a contiguous 1/8 of the list, and the tiles one XCD works on at
// the same time are neighbours that share halo rows and columns in its L2.
template <class T>
inline std::vector<T> xcd_order(const std::vector<T>& tiles) {
  const int nb = (int)tiles.size();
  std::vector<T> out(tiles.size());
  const int per = (nb + 7) / 8;
  const int full = nb - 8 * (per - 1);
  for (int w = 0; w < nb; ++w) {
    const int xcd = w % 8, k = w / 8;
    const int t = xcd < full ? xcd * per + k
                             : full * per + (xcd - full) * (per - 1) + k;
    out[w] = tiles[t];
  }
  return out;
}

// Blocks of the tile kernel: one per tile (the hardware schedules them), or,
// with LBPC_PERSISTENT=1, one per resident slot walking the list.
inline int tile_grid(int nwork, int prec, int bw) {
  const char* v = std::getenv("LBPC_PERSISTENT");
  if (!(v && std::atoi(v) != 0)) return nwork;
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess)
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount,
                                dev);
  const int waves = fp16_form(prec) ? 3 : 2;
  int per_cu = 4 * waves / (bw / 64);
  if (per_cu < 1) per_cu = 1;
  return nwork < cus * per_cu ? nwork : cus * per_cu;
}

// block widths (threads per block) the step kernels are built for; a strip
// is that many columns minus the 2 x 2 halo columns
inline bool valid_block_width(int bw) {
  return bw == 64 || bw == 128 || bw == 256 || bw == 512;
}

inline int env_int(const char* name, int dflt) {
  const char* v = std::getenv(name);
  return v ? std::atoi(v) : dflt;
}

// Blocks of the step kernel resident per CU: the waves-per-SIMD budget the
// kernel is compiled for (3 for the FP16 forms, 2 for the others) over the
// block's waves, capped by its LDS (5 rings x 5 fields, plus the g ring of
// the reduced-precision forms' two-row prefetch) against the CU's 160 KiB.
inline int blocks_per_cu(int precision, int bw) {
  const bool fp64 = precision == LBPC_FP64;
  const int by_waves = 4 * (fp16_form(precision) ? 3 : 2) / (bw / 64);
  const int lds = fp64 ? 25 * 8 * bw : 25 * 4 * bw + 27 * 4 * bw;
  const int by_lds = 160 * 1024 / lds;
  const int n = by_waves < by_lds ? by_waves : by_lds;
  return n < 1 ? 1 : n;
}

// Rows per tile for nbx strips: a tile's block marches rows + 4 row
// iterations, and the tiles run in ceil(tiles / slots) waves, so the time
// goes as waves x (rows + 4).  Minimised over rows >= 16 this prefers the
// tallest runs whose tile count just fits a whole number of waves (4096^2
// FP64 with 512-thread blocks: 147 rows, 252 tiles in one wave of 256
// slots, 16.26k MLUPS against 15.83k for 37 rows in 3.9 waves; the model
// ranks all ten heights measured there in order).
inline int fill_rows(int ny, int nbx, long long slots) {
  int best_rows = ny < 16 ? ny : 16;
  long long best = -1;
  for (int rows = best_rows; rows <= ny; ++rows) {
    const long long nby = (ny + rows - 1) / rows;
    const long long waves = (nbx * nby + slots - 1) / slots;
    const long long cost = waves * (rows + 4);
    if (best < 0 || cost < best) {
      best = cost;
      best_rows = rows;
    }
  }
  return best_rows;
}

// Strips holding a non-periodic x side; on the tile-list path they may run
// shorter row runs (He rows) than the others (H rows).
inline bool edge_strip(const StepParams& p, int bx) {
  return !p.perx && (bx == 0 || bx == p.nbx - 1);
}

// The tiles of one lattice as (0, bx, by, slot), row of runs by row of runs;
// slot numbers them in this order (their diagnostic records).
inline std::vector<std::array<int, 4>> tile_list(const StepParams& p) {
  const int ni = (p.ny + p.H - 1) / p.H, ne = (p.ny + p.He - 1) / p.He;
  const int nmax = ni > ne ? ni : ne;
  std::vector<std::array<int, 4>> t;
  for (int by = 0; by < nmax; ++by)
    for (int bx = 0; bx < p.nbx; ++bx)
      if (by < (edge_strip(p, bx) ? ne : ni))
        t.push_back({0, bx, by, (int)t.size()});
  return t;
}

// Default rows per tile of a single lattice for block width bw (rows_edge:
// the x-edge strips' runs, the same height by default): the wave-filling
// height of fill_rows for the device's CUs.  One exception: the FP32 forms
// on a non-periodic lattice (the boundary-capable tile kernel, 256-thread
// blocks, two per CU) run best at the height whose tiles fill three waves
// of slots exactly.  On a 4096^2 lattice walled on all four sides (17
// strips, 512 slots): FP32 29.5k MLUPS at 46 rows (1530 tiles) against
// 28.2k at 20, 27.6k at 38, 26.3k at 54 and 24.4k at 92; FP32 deviations
// 29.1k at 46 against 27.7k at 20 and 24.1k at 92.  FP16 deviations (three
// blocks per CU) run best at the one-wave height, 92 rows: 36.0k against
// 33.6k at 20.
inline void default_rows(const lbpc_config& c, bool tiled, int cus, int bw,
                         int& rows, int& rows_edge) {
  int nbx, W;
  strip_shape(c.nx, bw, balanced_strips(c.precision, bw), nbx, W);
  long long slots = (long long)cus * blocks_per_cu(c.precision, bw);
  if (tiled &&
      (c.precision == LBPC_FP32 || c.precision == LBPC_FP32_SHIFTED))
    slots *= 3;
  rows = rows_edge = fill_rows(c.ny, nbx, slots);
}

// Two steps per launch (lbpc_step2.hip), on request (LBPC_TWO_STEP=1): the
// 4-byte storage forms on periodic lattices of at least 16 x 16 nodes under
// the improved or the compromised thermal model, unless steady steps are
// replayed from a graph.  Off by default: at 4096^2 FP32 it ran 32.1k MLUPS
// against 34.1k for single steps (one wave per SIMD, latency-bound).  Blocks of 256 threads on strips of at most 246
// columns (5 halo columns per side), one block per CU (134 KiB of LDS), and
// the run height that fills whole waves of blocks, by the cost model of
// fill_rows with 12 extra row iterations per run.  Returns whether it is
// used; the tiling goes into q (nbx, W, nby, H, bw).
inline bool two_step_tiles(const lbpc_config& c, bool tiled, bool graph,
                           int cus, StepParams& q) {
  const bool form = c.precision == LBPC_FP32 ||
                    c.precision == LBPC_FP32_SHIFTED;
  const bool model = c.thermal_model == LBPC_THERMAL_IMPROVED ||
                     c.thermal_model == LBPC_THERMAL_COMPROMISED;
  if (!form || !model || tiled || graph || c.nx < 16 || c.ny < 16 ||
      env_int("LBPC_TWO_STEP", 0) == 0)
    return false;
  q.bw = 256;
  q.nbx = (c.nx + 245) / 246;
  q.W = (c.nx + q.nbx - 1) / q.nbx;
  int best_rows = c.ny < 16 ? c.ny : 16;
  long long best = -1;
  for (int rows = best_rows; rows <= c.ny; ++rows) {
    const long long nby = (c.ny + rows - 1) / rows;
    const long long waves = (q.nbx * nby + cus - 1) / cus;
    const long long cost = waves * (rows + 12);
    if (best < 0 || cost < best) {
      best = cost;
      best_rows = rows;
    }
  }
  q.H = best_rows;
  q.nby = (c.ny + q.H - 1) / q.H;
  return true;
}

// Default tile shape of a single lattice (LBPC_TILE_BW, LBPC_TILE_H and,
// with LBPC_TILE_H, LBPC_TILE_HE override it; lbpc_autotune and
// lbpc_set_tiles change it later).  512-thread blocks (8 waves, one
// block per CU at 2 waves per SIMD) read half the halo columns of
// 256-thread strips: at 4096^2 FP64 +3.8 % (+3.6 % with walls), periodic
// FP32 +5 %.  The FP32 forms on non-periodic lattices (the heavier
// boundary-capable kernel) keep 256: walled 4096^2 FP32 ran 26.9k MLUPS at
// 512 x 147 against 29.5k at 256 x 46.  So does the FP16-deviation form,
// compiled for three waves per SIMD: periodic 4096^2 0.357 ms per step at
// 256 x 92 against 0.476 at 512 x 32.
inline void default_tiles(const lbpc_config& c, bool tiled, int cus, int& bw,
                          int& rows, int& rows_edge) {
  const bool wide = c.precision == LBPC_FP64 ||
                    (!fp16_form(c.precision) && !tiled);
  bw = env_int("LBPC_TILE_BW", wide ? 512 : 256);
  if (!valid_block_width(bw)) bw = 256;
  // runs shorter than 4 rows are not supported (the tile list and its
  // workspace capacity assume at least 4): such a setting is ignored
  rows = env_int("LBPC_TILE_H", 0);
  if (rows >= 4) {
    rows_edge = env_int("LBPC_TILE_HE", rows);
    if (rows_edge < 4) rows_edge = rows;
  } else {
    default_rows(c, tiled, cus, bw, rows, rows_edge);
  }
}

// Transfers through the staging scratch `scr` (five fields of `stage` FP64
// values, stage >= 3 nx), chunk by chunk on stream s.  Stream order
// keeps each chunk's kernel ahead of the copy that refills the scratch.
// Each returns the first HIP error, with the failing call named in *what,
// after synchronising s.

// Initial fields (host rho, ux, uy, T of N nodes each) -> populations.
inline hipError_t stage_init(const StepParams& p, int prec, double* scr,
                             size_t stage, const double* const src[4],
                             hipStream_t s, const char** what) {
  const long long N = p.N;
  const long long C = (long long)stage * 5 / 4;
  hipError_t e = hipSuccess;
  for (long long i0 = 0; i0 < N && e == hipSuccess; i0 += C) {
    const long long cnt = std::min(C, N - i0);
    *what = "copy of the initial fields";
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
      e = hipMemcpyAsync(scr + k * cnt, src[k] + i0, cnt * sizeof(double),
                         hipMemcpyHostToDevice, s);
    if (e != hipSuccess) break;
    *what = "init kernel";
    e = lbpc::launch_init(p, prec, scr, i0, cnt, s);
  }
  if (e != hipSuccess) return e;
  *what = "synchronise";
  return hipStreamSynchronize(s);
}

// Fields rho, ux, uy, T at the current time level -> host arrays of N
// nodes (a NULL destination is skipped), band by band of rows.
inline hipError_t stage_fields(const StepParams& p, int prec, double* scr,
                               size_t stage, double* const dst[4],
                               hipStream_t s, const char** what) {
  const int R = (int)std::min(stage / (size_t)p.nx - 2, (size_t)p.ny);
  hipError_t e = hipSuccess;
  for (int y0 = 0; y0 < p.ny && e == hipSuccess; y0 += R) {
    const int nr = std::min(R, p.ny - y0);
    const size_t m = (size_t)(nr + 2) * p.nx;
    *what = "macro kernels";
    e = lbpc::launch_macro(p, prec, scr, y0, nr, s);
    *what = "copy of the fields";
    for (int k = 0; k < 4 && e == hipSuccess; ++k)
      if (dst[k])
        e = hipMemcpyAsync(dst[k] + (size_t)y0 * p.nx, scr + k * m + p.nx,
                           (size_t)nr * p.nx * sizeof(double),
                           hipMemcpyDeviceToHost, s);
  }
  if (e != hipSuccess) return e;
  *what = "synchronise";
  return hipStreamSynchronize(s);
}

// One FP64 array of N nodes of the checkpoint, device -> host (out) or
// host -> device (!out): which 0-8 / 9-17 the canonical f / g populations,
// which < 0 the history array at p.phi.
inline hipError_t stage_state(const StepParams& p, int prec, int which,
                              bool out, double* scr, size_t stage,
                              double* host, hipStream_t s, const char** what) {
  const long long N = p.N;
  const long long C = (long long)stage * 5;
  hipError_t e = hipSuccess;
  for (long long i0 = 0; i0 < N && e == hipSuccess; i0 += C) {
    const long long cnt = std::min(C, N - i0);
    if (out) {
      *what = which < 0 ? "history copy kernel" : "canonical-state kernel";
      e = which < 0 ? lbpc::launch_phi_out(p, prec, scr, i0, cnt, s)
                    : lbpc::launch_canon(p, prec, which, scr, i0, cnt, s);
      if (e != hipSuccess) break;
      *what = "state copy";
      e = hipMemcpyAsync(host + i0, scr, cnt * sizeof(double),
                         hipMemcpyDeviceToHost, s);
    } else {
      *what = "state copy";
      e = hipMemcpyAsync(scr, host + i0, cnt * sizeof(double),
                         hipMemcpyHostToDevice, s);
      if (e != hipSuccess) break;
      *what = which < 0 ? "history load kernel" : "state load kernel";
      e = which < 0 ? lbpc::launch_phi_in(p, prec, scr, i0, cnt, s)
                    : lbpc::launch_load(p, prec, which, scr, i0, cnt, s);
    }
  }
  if (e != hipSuccess) return e;
  *what = "synchronise";
  return hipStreamSynchronize(s);
}

}  // namespace lbpc_host

