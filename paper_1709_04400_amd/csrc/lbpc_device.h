// lbpc_device.h -- device-side building blocks of the gfx950 step kernels:
// kernel parameters, storage-precision traits, the Peng-Robinson EOS of
// Eq. (56), the ghost rule of the non-periodic sides and the MRT transforms.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lbpc {

constexpr int Q = 9;
constexpr int HALO = 2;         // columns of halo on each side of a strip
constexpr int RING = 5;         // rows held in the LDS ring buffers

enum { BC_PERIODIC = 0, BC_WALL = 1, BC_OPEN = 2 };
enum { GH_INSIDE = 0, GH_WALL = 1, GH_OPEN = 2 };

// Everything a step kernel needs, passed by value.
struct StepParams {
  // lattice and tiling
  int nx, ny;
  int perx, pery;          // 1 if that axis is periodic
  int bc[4];               // side kinds x-, x+, y-, y+
  int W, H;                // interior columns / rows per block
  int He;                  // rows per block of the x-edge strips when the x
                           // sides are not periodic (tile-list kernel)
  int nbx, nby;            // blocks along x and y
  int bw;                  // threads per block (strip width incl. halo)
  int xcd_order;           // 1: blocks of one XCD take x-adjacent strips
  int hot_x0, hot_x1;
  double T_bc[4], T_hot;
  // EOS (Eq. 56) and flow model
  double a, b, R, Tc, kappa;
  double G, sigma;
  double gx, gy, rho_ave;
  double s_f[9];
  // thermal model
  double s_g[9];
  double cv, lambda0, chi, k_th;
  int lambda_mode, improved;
  int gc;                  // Gong-Cheng model (BGK, Eqs. 12-14)
  int bgk;                 // BGK form of the improved model (Eq. 33)
  double bgk_itau;         // its 1/tau_g
  double bgk_cfac;         // (1 - 1/(2 tau_g)) / c_s^2 of Eq. (31)
  double wg0, wg1, wg2;    // rest equilibrium of g per unit T: rest, axis,
                           // diagonal (Eq. 53, or Eq. 14 for Gong-Cheng)
  double gc_ta, gc_tb;     // Gong-Cheng: tau_g = gc_ta / rho + gc_tb
  // wall wetting: a ghost across a wall enters the interaction force with
  // psi of the virtual density (1 + wet_amp) rho_n - wet_shift, clamped to
  // [0, 0.9/b], at T_n of its nearest node n (wet = 0: psi_n itself)
  int wet;
  double wet_amp, wet_shift;
  // derived on the host: 1/Tc, 2/G, 1/c_V, lambda0/c_V and the sigma terms
  // 12 sigma G^2 / (1/s_f[k] - 1/2), k = 1, 2 (|F_m|^2/psi^2 = G^2 |s|^2)
  double inv_Tc, two_over_G, inv_cv, lam_over_cv, sig1, sig2;
  // storage shift (rho_ref, T_ref of the shifted forms)
  double rho_ref, T_ref;
  // coexistence densities of the liquid-area diagnostic
  double rho_v, rho_l;
  // state flags
  int fresh;      // 1: the input buffer holds pre-collision f(t) (no pull)
  int phi_valid;  // 0: first step, phi_prev := phi
  // buffers
  const void* fin;  // [ny][9][nx] input f (post-collision f*(t-1) or fresh f(t))
  const void* gin;
  void* fout;       // [ny][9][nx] output f*(t)
  void* gout;
  void* phi;        // [N] phi(t-1) (compute precision); for the BGK form
                    // followed by [N] T v_x and [N] T v_y of step t-1
  void* phi_out;    // the same for step t; the same arrays except while
                    // the autotuner times steps
  const void* rin;  // FP16 deviation form only: the rest populations of the
  void* rout;       // input / output buffer in FP32, [N] f_0 then [N] g_0
                    // (deviations; direction 0 of the FP16 arrays is unused)
  long long N;      // nx * ny
  int* bad;         // set to 1 when a step meets an invalid node state
                    // (host-mapped memory, read by the host without waiting)
};

// ------------------------------------------------------- precision traits

// Accesses to the distribution buffers go through global (address space 1)
// pointers: they are device memory, and a pointer read from a parameter
// table would otherwise be accessed with flat instructions.
template <class T> using Gbl = __attribute__((address_space(1))) T;
template <class T>
__device__ __forceinline__ const Gbl<T>* gbl(const T* p) {
  return (const Gbl<T>*)p;
}
template <class T>
__device__ __forceinline__ Gbl<T>* gbl(T* p) { return (Gbl<T>*)p; }

// S: storage type; C: compute type; R: register image of a loaded value.
// A pulled value is kept as R until it is used, so a load can stay in
// flight across the work between its issue and its use; cvt() turns it into
// a compute value.
template <int P> struct Prec;
// `paired`: f and g of a direction are stored side by side, one (f, g) word
// per direction and node, since both stream from the same node: one access
// per lane moves both.  FP64 keeps separate f and g arrays (the 16-byte pair
// gained 2 % on its memory schedule, less than the registers it would cost
// to hold f* for the pair).
template <> struct Prec<0> {  // FP64 storage and arithmetic
  using S = double;
  using C = double;
  using R = double;
  static constexpr bool shift = false;
  static constexpr bool paired = false;
  __device__ static R ldr(const S* p, long long i) { return gbl(p)[i]; }
  __device__ static C cvt(R v) { return v; }
  __device__ static C ld(const S* p, long long i) { return gbl(p)[i]; }
  __device__ static void st(S* p, long long i, C v) { gbl(p)[i] = v; }
};
// FP32 storage and arithmetic; the (f, g) pair of a direction is 8 bytes.
template <> struct Prec<1> {
  using S = float;
  using C = float;
  using R = float;
  static constexpr bool shift = false;
  static constexpr bool paired = true;
  __device__ static C cvt(R v) { return v; }
};
// FP32 deviations from the rest equilibrium, in (f, g) pairs as FP32.
template <> struct Prec<2> {
  using S = float;
  using C = float;
  using R = float;
  static constexpr bool shift = true;
  static constexpr bool paired = true;
  __device__ static C cvt(R v) { return v; }
};
// FP16 deviations, FP32 arithmetic.  f and g of one direction share a
// 32-bit word (binary16 f in the low half, g in the high half): they stream
// from the same node, so one 4-byte access per lane moves both, where
// separate arrays would take two 2-byte accesses.
template <> struct Prec<3> {
  using S = unsigned int;  // the (f, g) word
  using C = float;
  using R = unsigned int;  // the word as loaded
  static constexpr bool shift = true;
  static constexpr bool paired = true;
  __device__ static R ldr(const S* p, long long i) { return gbl(p)[i]; }
  __device__ static C cvt(R v) {  // f, the low half
    return __half2float(__ushort_as_half((unsigned short)v));
  }
  __device__ static C cvt_hi(R v) {  // g, the high half
    return __half2float(__ushort_as_half((unsigned short)(v >> 16)));
  }
};
// FP16 deviations from node-local references, FP32 arithmetic.  Every node
// keeps a reference word in its direction-0 slot: binary16 rho_ref (low
// half) and T_ref (high half), the density and temperature it had when the
// word was stored.  The (f, g) word of direction a of node x holds
// f*_a - w_a rho_ref and g*_a - wg_a T_ref against the reference of the node
// that pulls it: x + e_a, or x itself where e_a crosses a wall.  A puller
// then adds its own reference (one 4-byte load per node) and the stored
// values are the velocity and non-equilibrium parts only, which binary16
// resolves in the liquid as finely as in the vapour.  The rest populations
// are FP32 full values.  (Across an open side the clamped source's value
// was stored against its interior neighbour's reference, which the puller
// reads there.)
template <> struct Prec<4> {
  using S = unsigned int;
  using C = float;
  using R = unsigned int;
  static constexpr bool shift = false;
  static constexpr bool paired = true;
  __device__ static R ldr(const S* p, long long i) { return gbl(p)[i]; }
  __device__ static C cvt(R v) {
    return __half2float(__ushort_as_half((unsigned short)v));
  }
  __device__ static C cvt_hi(R v) {
    return __half2float(__ushort_as_half((unsigned short)(v >> 16)));
  }
};

// reference word of the node-referenced FP16 form: binary16 rho | T << 16
// (round to nearest even)
__device__ __forceinline__ unsigned int ref_word(float rho, float T) {
  return (unsigned int)__half_as_ushort(__float2half_rn(rho)) |
         ((unsigned int)__half_as_ushort(__float2half_rn(T)) << 16);
}

// D2Q9 weights (shift of f, Eq. 14) and the rest equilibrium of g of the
// lattice's thermal model (side rules and shift of g)
__device__ __forceinline__ double w_lat(int a) {
  return a == 0 ? 4.0 / 9.0 : (a < 5 ? 1.0 / 9.0 : 1.0 / 36.0);
}
__device__ __forceinline__ double w_rest(const StepParams& p, int a) {
  return a == 0 ? p.wg0 : (a < 5 ? p.wg1 : p.wg2);
}

// 1/x and sqrt(x): IEEE division and square root in FP64; in the FP32
// arithmetic of the reduced-precision forms the hardware's reciprocal and
// square root (each within 1 ulp), which save the ~10 and ~14 instructions of
// the correctly rounded forms per use in kernels bound by instruction issue
__device__ __forceinline__ double recip(double x) { return 1.0 / x; }
__device__ __forceinline__ float recip(float x) {
  return __builtin_amdgcn_rcpf(x);
}
__device__ __forceinline__ float fsqrt(float x) {
  return __builtin_amdgcn_sqrtf(x);
}

// ---------------------------------------------------------- EOS, Eq. (56)

__device__ __forceinline__ double pr_p(const StepParams& p, double rho,
                                       double T) {
  double s = 1.0 + p.kappa * (1.0 - sqrt(T / p.Tc));
  double th = s * s;
  return rho * p.R * T / (1.0 - p.b * rho) -
         p.a * th * rho * rho / (1.0 + 2.0 * p.b * rho - p.b * p.b * rho * rho);
}

__device__ __forceinline__ double pr_dpdT(const StepParams& p, double rho,
                                          double T) {
  double s = 1.0 + p.kappa * (1.0 - sqrt(T / p.Tc));
  double dth = 2.0 * s * (-p.kappa) * (0.5 / sqrt(T * p.Tc));
  return rho * p.R / (1.0 - p.b * rho) -
         p.a * dth * rho * rho /
             (1.0 + 2.0 * p.b * rho - p.b * p.b * rho * rho);
}

// psi = sqrt(2 (p_EOS - rho c_s^2) / G) with c = 1, evaluated in FP64 (the
// difference cancels strongly in the liquid)
__device__ __forceinline__ double pseudo_psi(const StepParams& p, double rho,
                                             double T) {
  double psi2 = 2.0 * (pr_p(p, rho, T) - rho * (1.0 / 3.0)) / p.G;
  return sqrt(psi2 > 0.0 ? psi2 : 0.0);
}

// psi of a ghost across a wall (wetting): the virtual density of the ghost's
// nearest lattice node n, (1 + wet_amp) rho_n - wet_shift clamped to
// [0, 0.9/b], at T_n
__device__ __forceinline__ double wall_psi(const StepParams& p, double rho_n,
                                           double T_n) {
  double rw = (1.0 + p.wet_amp) * rho_n - p.wet_shift;
  rw = rw < 0.0 ? 0.0 : (rw > 0.9 / p.b ? 0.9 / p.b : rw);
  return pseudo_psi(p, rw, T_n);
}

// ------------------------------------------------------------ ghost rule

__device__ __forceinline__ double side_T(const StepParams& p, int side,
                                         int col) {
  if (side == 2 && col >= p.hot_x0 && col < p.hot_x1) return p.T_hot;
  return p.T_bc[side];
}

struct Ghost {
  int kind;    // GH_INSIDE, GH_WALL, GH_OPEN
  int x, y;    // node after periodic wrap (inside) or clamping (ghost)
  double T;    // ghost temperature
};

// Resolve an unwrapped lattice position: wrap periodic axes, clamp the
// others, and classify (a wall wins over an open side; the y side gives T at
// corners).
__device__ __forceinline__ Ghost resolve(const StepParams& p, int x, int y) {
  Ghost g;
  int xs = -1, ys = -1;
  if (x < 0 || x >= p.nx) {
    int side = x < 0 ? 0 : 1;
    if (p.perx) {
      x = x < 0 ? x + p.nx : x - p.nx;
    } else {
      xs = side;
      x = x < 0 ? 0 : p.nx - 1;
    }
  }
  if (y < 0 || y >= p.ny) {
    int side = y < 0 ? 2 : 3;
    if (p.pery) {
      y = y < 0 ? y + p.ny : y - p.ny;
    } else {
      ys = side;
      y = y < 0 ? 0 : p.ny - 1;
    }
  }
  g.x = x;
  g.y = y;
  g.T = 0.0;
  if (xs < 0 && ys < 0) {
    g.kind = GH_INSIDE;
  } else {
    bool wall = (ys >= 0 && p.bc[ys] == BC_WALL) ||
                (xs >= 0 && p.bc[xs] == BC_WALL);
    g.kind = wall ? GH_WALL : GH_OPEN;
    g.T = ys >= 0 ? side_T(p, ys, x) : side_T(p, xs, x);
  }
  return g;
}

// Shifts of the shifted storage forms: f is stored as f_a - w_a rho_ref and
// g as g_a - wg_a T_ref.  Three f and three g shifts (rest, axis, diagonal)
// are distinct; zero for the plain forms.
template <int P>
struct Shift {
  using C = typename Prec<P>::C;
  C f0, f1, f2, g0, g1, g2;
  __device__ __forceinline__ explicit Shift(const StepParams& p) {
    if constexpr (Prec<P>::shift) {
      f0 = C(w_lat(0) * p.rho_ref);
      f1 = C(w_lat(1) * p.rho_ref);
      f2 = C(w_lat(5) * p.rho_ref);
      g0 = C(p.wg0 * p.T_ref);
      g1 = C(p.wg1 * p.T_ref);
      g2 = C(p.wg2 * p.T_ref);
    } else {
      f0 = f1 = f2 = g0 = g1 = g2 = C(0);
    }
  }
  __device__ __forceinline__ C f(int a) const {
    if constexpr (!Prec<P>::shift) return C(0);
    return a == 0 ? f0 : (a < 5 ? f1 : f2);
  }
  __device__ __forceinline__ C g(int a) const {
    if constexpr (!Prec<P>::shift) return C(0);
    return a == 0 ? g0 : (a < 5 ? g1 : g2);
  }
};

// ------------------------------------------------------------- the pull
// f_a(x, t) = f*_a(x - e_a, t - 1), and likewise g, at lattice node (x, y),
// with the side rules at edge nodes: across a wall halfway bounce-back for f
// and anti-bounce-back g_a = -g*_abar + 2 wg_a T_wall for g; across an open
// side f_a = f*_a(clamped source), g_a = wg_a T_side.  A wall wins over an
// open side at a corner and the y side gives the temperature there.  With
// p.fresh the buffers hold f(t), g(t) themselves and are read in place.
//
// The pull is split in two so that its loads can be issued a row ahead:
//   pull_raw  issues the loads.  Source rows / columns are clamped on
//             non-periodic axes, and a wave holding an edge node takes, for
//             each wall-crossing direction, f*_abar and g*_abar of the node
//             itself (branch-free inside the wave).
//   cook_f,   turn the raw registers into unshifted compute values (the
//   cook_g    node-referenced FP16 form adds each value's reference); cook_g
//             then applies the value rules of g at edge nodes (again only
//             in waves that hold one).

// Distribution buffers interleave the rows of the nine direction arrays,
// [ny][9][nx]: value a of node (x, y) is element dix(nx, a, y, x).  A tile
// row then reads and writes one contiguous stretch of each buffer (plus the
// neighbour rows of the pull) instead of nine arrays a lattice apart, which
// the HBM serves faster than the same bytes spread over 18 streams.
__device__ __forceinline__ long long dix(int nx, int a, long long y, int x) {
  return (y * Q + a) * nx + x;
}

constexpr int EXs[Q] = {0, 1, 0, -1, 0, 1, -1, -1, 1};
constexpr int EYs[Q] = {0, 0, 1, 0, -1, 1, 1, -1, -1};
constexpr int OPs[Q] = {0, 3, 4, 1, 2, 7, 8, 5, 6};

// Which sides the pull of node (x, y) crosses.
struct EdgeSides {
  bool o0, o1, o2, o3;  // x-, x+, y-, y+
  __device__ __forceinline__ EdgeSides(const StepParams& p, int x, int y,
                                       bool gen) {
    const bool clx = gen && !p.perx, cly = gen && !p.pery;
    o0 = clx && x == 0;
    o1 = clx && x == p.nx - 1;
    o2 = cly && y == 0;
    o3 = cly && y == p.ny - 1;
  }
  __device__ __forceinline__ bool any() const { return o0 || o1 || o2 || o3; }
  // direction a crosses a side / a wall
  __device__ __forceinline__ bool ox(int a) const {
    return EXs[a] > 0 ? o0 : (EXs[a] < 0 ? o1 : false);
  }
  __device__ __forceinline__ bool oy(int a) const {
    return EYs[a] > 0 ? o2 : (EYs[a] < 0 ? o3 : false);
  }
  __device__ __forceinline__ bool wall(const StepParams& p, int a) const {
    return (ox(a) && p.bc[EXs[a] > 0 ? 0 : 1] == BC_WALL) ||
           (oy(a) && p.bc[EYs[a] > 0 ? 2 : 3] == BC_WALL);
  }
};

// Neighbour column x + dx: wrapped on a periodic x axis, clamped otherwise.
__device__ __forceinline__ int wrap_or_clamp(int v, int n, bool periodic) {
  if (v < 0) return periodic ? v + n : 0;
  if (v >= n) return periodic ? v - n : n - 1;
  return v;
}

template <int P, bool GEN>
__device__ __forceinline__ void pull_raw(
    const StepParams& p, const typename Prec<P>::S* __restrict__ fin,
    const typename Prec<P>::S* __restrict__ gin, int x, int y,
    typename Prec<P>::R fr[Q], typename Prec<P>::R gr[Q]) {
  using Tr = Prec<P>;
  const int nx = p.nx, ny = p.ny;
  // element offset of each direction's source; one set of loads serves
  // every case below, so the loads never sit in divergent branches
  long long off[Q];
  if (p.fresh) {
#pragma unroll
    for (int a = 0; a < Q; ++a) off[a] = dix(nx, a, y, x);
  } else {
    const int xm = wrap_or_clamp(x - 1, nx, !GEN || p.perx);
    const int xp = wrap_or_clamp(x + 1, nx, !GEN || p.perx);
    const int ym = wrap_or_clamp(y - 1, ny, !GEN || p.pery);
    const int yp = wrap_or_clamp(y + 1, ny, !GEN || p.pery);
    // source of direction a is x - e_a
    const int ys[Q] = {y, y, ym, y, yp, ym, ym, yp, yp};
    const int xs[Q] = {x, xm, x, xp, x, xm, xp, xp, xm};
#pragma unroll
    for (int a = 0; a < Q; ++a) off[a] = dix(nx, a, ys[a], xs[a]);
    if (GEN) {
      const EdgeSides e(p, x, y, true);
      if (__builtin_amdgcn_ballot_w64(e.any()) != 0) {
#pragma unroll
        for (int a = 1; a < Q; ++a)
          if (e.wall(p, a)) off[a] = dix(nx, OPs[a], y, x);
      }
    }
  }
  if constexpr (P == 3) {
    // FP16 deviation form: one (f, g) word per direction, held in both fr
    // and gr (cook_f takes its low half, cook_g its high half); the rest
    // populations are an FP32 (f_0, g_0) pair per node, one 8-byte load
    const long long o = (long long)y * nx + x;
    const unsigned long long r =
        gbl(static_cast<const unsigned long long*>(p.rin))[o];
    fr[0] = (unsigned int)r;
    gr[0] = (unsigned int)(r >> 32);
#pragma unroll
    for (int a = 1; a < Q; ++a) fr[a] = gr[a] = Tr::ldr(fin, off[a]);
  } else if constexpr (P == 4) {
    // node-referenced FP16 form: the (f, g) words in fr, the rest pair in
    // fr[0] / gr[0], and in gr[1..8] the reference the values were stored
    // against: the node's own (cook_f replaces it across an open side)
    const long long o = (long long)y * nx + x;
    const unsigned long long r =
        gbl(static_cast<const unsigned long long*>(p.rin))[o];
    fr[0] = (unsigned int)r;
    gr[0] = (unsigned int)(r >> 32);
    const unsigned int own = Tr::ldr(fin, dix(nx, 0, y, x));
#pragma unroll
    for (int a = 1; a < Q; ++a) {
      fr[a] = Tr::ldr(fin, off[a]);
      gr[a] = own;
    }
  } else if constexpr (Tr::paired) {
    // FP32 forms: one 8-byte (f, g) pair per direction
    const Gbl<unsigned long long>* w =
        gbl(reinterpret_cast<const unsigned long long*>(fin));
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const unsigned long long v = w[off[a]];
      fr[a] = __uint_as_float((unsigned int)v);
      gr[a] = __uint_as_float((unsigned int)(v >> 32));
    }
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      fr[a] = Tr::ldr(fin, off[a]);
      gr[a] = Tr::ldr(gin, off[a]);
    }
  }
}

// Raw register image -> compute value of direction a of f (G = false) or g
// (G = true); in the FP16 deviation form the rest population is an FP32
// image and the others a half of the (f, g) word.
template <int P, bool G>
__device__ __forceinline__ typename Prec<P>::C raw_value(
    const typename Prec<P>::R v, int a) {
  if constexpr (P == 3) {
    if (a == 0) return __uint_as_float(v);
    return G ? Prec<3>::cvt_hi(v) : Prec<3>::cvt(v);
  } else {
    return Prec<P>::cvt(v);
  }
}

// Store of the nine post-collision values d[a] of one node into separate
// arrays (FP64): element dix(nx, a, y, x) of buf.
template <int P>
__device__ __forceinline__ void store_node(typename Prec<P>::S* buf, int nx,
                                           long long y, int x,
                                           const typename Prec<P>::C d[Q]) {
  static_assert(!Prec<P>::paired, "paired forms store (f, g) pairs");
#pragma unroll
  for (int a = 0; a < Q; ++a) gbl(buf)[dix(nx, a, y, x)] = d[a];
}

// FP16 deviation form, one distribution of a node: the binary16 bits of
// d[1..8] (round to nearest even), each in the low half of h[a], and the
// rest value d[0] less the rounding errors of the other eight, so that the
// node's stored sum is the computed sum to FP32 rounding and biased rounding
// of near-constant populations does not drift the mass (or sum T) of the
// lattice.
__device__ __forceinline__ void half_node(const float d[Q], unsigned int h[Q],
                                          float& rest) {
  float err = 0.0f;
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const __half v = __float2half_rn(d[a]);
    h[a] = __half_as_ushort(v);
    err += __half2float(v) - d[a];
  }
  rest = d[0] - err;
}

// Paired forms: f* of a node (storage form) as the 32-bit images it is
// stored with, held until g* of the node is ready: FP32 bits, or in the
// FP16 deviation form binary16 bits for directions 1-8 and the FP32 bits of
// the compensated rest value for direction 0.
template <int P>
__device__ __forceinline__ void pack_f(const float d[Q], unsigned int h[Q]) {
  static_assert(Prec<P>::paired, "pairs only");
  if constexpr (P == 3) {
    float rest;
    half_node(d, h, rest);
    h[0] = __float_as_uint(rest);
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) h[a] = __float_as_uint(d[a]);
  }
}

// Node-referenced FP16 form: as half_node, with the value of direction a
// taken relative to r[a] (its reference times its weight).
__device__ __forceinline__ void half_node_ref(const float d[Q],
                                              const float r[Q],
                                              unsigned int h[Q],
                                              float& rest) {
  float err = 0.0f;
#pragma unroll
  for (int a = 1; a < Q; ++a) {
    const float dv = d[a] - r[a];
    const __half v = __float2half_rn(dv);
    h[a] = __half_as_ushort(v);
    err += __half2float(v) - dv;
  }
  rest = d[0] - err;
}

// binary16 rounding of a reference value, as the puller reads it back
__device__ __forceinline__ float ref_round(float v) {
  return __half2float(__float2half_rn(v));
}

// Node-referenced FP16 form: f* of a node as the images it is stored with
// (as pack_f), each direction a >= 1 less w_a rr[a], rr[a] the rho_ref
// (a binary16 value) of the node that pulls it.
__device__ __forceinline__ void pack_f_local(const float d[Q],
                                             const float rr[Q],
                                             unsigned int h[Q]) {
  float wr[Q];
  wr[0] = 0.0f;
#pragma unroll
  for (int a = 1; a < Q; ++a) wr[a] = float(w_lat(a)) * rr[a];
  float rest;
  half_node_ref(d, wr, h, rest);
  h[0] = __float_as_uint(rest);
}

// Node-referenced FP16 form: store of node (y, x) from f* as packed by
// pack_f_local and g* (FP32), each direction a >= 1 less wg_a tr[a], tr[a]
// the T_ref of the node that pulls it: its own reference word `own` into
// direction 0, the (f, g) words of directions 1-8 and the FP32 rest pair.
__device__ __forceinline__ void store_pairs_local(
    const StepParams& p, unsigned int* buf, void* rest, int nx, long long y,
    int x, const unsigned int hf[Q], const float go[Q], const float tr[Q],
    unsigned int own) {
  float wt[Q];
  wt[0] = 0.0f;
#pragma unroll
  for (int a = 1; a < Q; ++a) wt[a] = float(w_rest(p, a)) * tr[a];
  unsigned int hg[Q];
  float rg;
  half_node_ref(go, wt, hg, rg);
  gbl(buf)[dix(nx, 0, y, x)] = own;
#pragma unroll
  for (int a = 1; a < Q; ++a)
    gbl(buf)[dix(nx, a, y, x)] =
        __builtin_amdgcn_perm(hg[a], hf[a], 0x05040100u);
  gbl(static_cast<unsigned long long*>(rest))[y * nx + x] =
      (unsigned long long)hf[0] |
      ((unsigned long long)__float_as_uint(rg) << 32);
}

// Paired forms: store of node (y, x) from f* as packed by pack_f and g*
// (storage form).  FP32: the 8-byte word f | g << 32 of each direction.
// FP16 deviations: the word hf | hg << 16 of directions 1-8 in buf and the
// FP32 pair (rest_f, rest_g) in rest.
template <int P>
__device__ __forceinline__ void store_pairs(typename Prec<P>::S* buf,
                                            void* rest, int nx, long long y,
                                            int x, const unsigned int hf[Q],
                                            const float go[Q]) {
  static_assert(Prec<P>::paired, "pairs only");
  if constexpr (P == 3) {
    unsigned int hg[Q];
    float rg;
    half_node(go, hg, rg);
    // one byte permute per word: the low halves of hf[a] and hg[a]
#pragma unroll
    for (int a = 1; a < Q; ++a)
      gbl(buf)[dix(nx, a, y, x)] =
          __builtin_amdgcn_perm(hg[a], hf[a], 0x05040100u);
    gbl(static_cast<unsigned long long*>(rest))[y * nx + x] =
        (unsigned long long)hf[0] |
        ((unsigned long long)__float_as_uint(rg) << 32);
  } else {
    Gbl<unsigned long long>* w =
        gbl(reinterpret_cast<unsigned long long*>(buf));
#pragma unroll
    for (int a = 0; a < Q; ++a)
      w[dix(nx, a, y, x)] = (unsigned long long)hf[a] |
                            ((unsigned long long)__float_as_uint(go[a]) << 32);
  }
}

template <int P, bool GEN>
__device__ __forceinline__ void cook_f(const StepParams& p, const Shift<P>& sh,
                                       int x, int y,
                                       const typename Prec<P>::R fr[Q],
                                       const typename Prec<P>::R gr[Q],
                                       typename Prec<P>::C f[Q]) {
  if constexpr (P == 4) {
    f[0] = __uint_as_float(fr[0]);
#pragma unroll
    for (int a = 1; a < Q; ++a)
      f[a] = Prec<4>::cvt(fr[a]) + float(w_lat(a)) * Prec<4>::cvt(gr[a]);
    const bool open = p.bc[0] == BC_OPEN || p.bc[1] == BC_OPEN ||
                      p.bc[2] == BC_OPEN || p.bc[3] == BC_OPEN;
    if (GEN && !p.fresh && open) {
      // across an open side the value comes from the clamped source, whose
      // puller is its neighbour x + e_a inside the lattice: the value was
      // stored against that node's reference, read here (waves with an
      // edge node of a lattice with an open side only: the load is waited
      // for at once, with the row prefetch in flight)
      const EdgeSides e(p, x, y, true);
      if (__builtin_amdgcn_ballot_w64(e.any()) != 0) {
        const Gbl<unsigned int>* w =
            gbl(static_cast<const unsigned int*>(p.fin));
#pragma unroll
        for (int a = 1; a < Q; ++a) {
          const bool ox = e.ox(a), oy = e.oy(a);
          if ((ox || oy) && !e.wall(p, a)) {
            int xd = ox ? x + EXs[a] : x, yd = oy ? y + EYs[a] : y;
            xd = xd < 0 ? 0 : (xd >= p.nx ? p.nx - 1 : xd);
            yd = yd < 0 ? 0 : (yd >= p.ny ? p.ny - 1 : yd);
            f[a] = Prec<4>::cvt(fr[a]) +
                   float(w_lat(a)) * Prec<4>::cvt(w[dix(p.nx, 0, yd, xd)]);
          }
        }
      }
    }
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if constexpr (Prec<P>::shift)
        f[a] = raw_value<P, false>(fr[a], a) + sh.f(a);
      else
        f[a] = Prec<P>::cvt(fr[a]);
    }
  }
}

template <int P, bool GEN>
__device__ __forceinline__ void cook_g(const StepParams& p, const Shift<P>& sh,
                                       int x, int y,
                                       const typename Prec<P>::R fr[Q],
                                       const typename Prec<P>::R gr[Q],
                                       typename Prec<P>::C g[Q]) {
  using C = typename Prec<P>::C;
  if constexpr (P == 4) {
    g[0] = __uint_as_float(gr[0]);
#pragma unroll
    for (int a = 1; a < Q; ++a)
      g[a] = Prec<4>::cvt_hi(fr[a]) +
             float(w_rest(p, a)) * Prec<4>::cvt_hi(gr[a]);
  } else {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      if constexpr (Prec<P>::shift)
        g[a] = raw_value<P, true>(gr[a], a) + sh.g(a);
      else
        g[a] = Prec<P>::cvt(gr[a]);
    }
  }
  if (GEN && !p.fresh) {
    const EdgeSides e(p, x, y, true);
    const bool edge = __builtin_amdgcn_ballot_w64(e.any()) != 0;
    // a row away from the y sides takes only the directions arriving across
    // an x side, at that side's temperature
    const bool xonly = !(e.o2 || e.o3);
    if (edge && xonly) {
      const bool w0 = p.bc[0] == BC_WALL, w1 = p.bc[1] == BC_WALL;
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        if (EXs[a] == 0) continue;
        const bool ox = EXs[a] > 0 ? e.o0 : e.o1;
        const bool wall = ox && (EXs[a] > 0 ? w0 : w1);
        const C wT = C(w_rest(p, a)) * C(p.T_bc[EXs[a] > 0 ? 0 : 1]);
        g[a] = wall ? C(2) * wT - g[a] : (ox ? wT : g[a]);
      }
    } else if (edge) {
      const int xm = wrap_or_clamp(x - 1, p.nx, p.perx);
      const int xp = wrap_or_clamp(x + 1, p.nx, p.perx);
#pragma unroll
      for (int a = 1; a < Q; ++a) {
        const bool ox = e.ox(a), oy = e.oy(a), wall = e.wall(p, a);
        // source column for the hot-spot test of the y- side; temperatures
        // selected in the compute type
        const int col = EXs[a] > 0 ? xm : (EXs[a] < 0 ? xp : x);
        const C Ty = EYs[a] > 0 ? (col >= p.hot_x0 && col < p.hot_x1
                                       ? C(p.T_hot)
                                       : C(p.T_bc[2]))
                                : C(p.T_bc[3]);
        const C wT =
            C(w_rest(p, a)) * (oy ? Ty : C(p.T_bc[EXs[a] > 0 ? 0 : 1]));
        g[a] = wall ? C(2) * wT - g[a] : ((ox || oy) ? wT : g[a]);
      }
    }
  }
}

// Whole pull in one call (the auxiliary kernels).
template <int P, bool GEN>
__device__ __forceinline__ void pull_node(
    const StepParams& p, const typename Prec<P>::S* __restrict__ fin,
    const typename Prec<P>::S* __restrict__ gin, int x, int y,
    const Shift<P>& sh,
    typename Prec<P>::C fn[Q], typename Prec<P>::C gn[Q]) {
  typename Prec<P>::R fr[Q], gr[Q];
  pull_raw<P, GEN>(p, fin, gin, x, y, fr, gr);
  cook_f<P, GEN>(p, sh, x, y, fr, gr, fn);
  cook_g<P, GEN>(p, sh, x, y, fr, gr, gn);
}

// ------------------------------------------------------- MRT transforms
// M: rows (rho, e, eps, jx, qx, jy, qy, pxx, pxy) over the D2Q9 order
// 0 rest, 1 +x, 2 +y, 3 -x, 4 -y, 5 (+,+), 6 (-,+), 7 (-,-), 8 (+,-).

template <class C>
__device__ __forceinline__ void to_moments(const C f[9], C m[9]) {
  C sa = f[1] + f[2] + f[3] + f[4];
  C sd = f[5] + f[6] + f[7] + f[8];
  C dx1 = f[1] - f[3], dy1 = f[2] - f[4];
  C dxd = f[5] - f[6] - f[7] + f[8];
  C dyd = f[5] + f[6] - f[7] - f[8];
  m[0] = f[0] + sa + sd;
  m[1] = -C(4) * f[0] - sa + C(2) * sd;
  m[2] = C(4) * f[0] - C(2) * sa + sd;
  m[3] = dx1 + dxd;
  m[4] = -C(2) * dx1 + dxd;
  m[5] = dy1 + dyd;
  m[6] = -C(2) * dy1 + dyd;
  m[7] = f[1] - f[2] + f[3] - f[4];
  m[8] = f[5] - f[6] + f[7] - f[8];
}

// f = M^-1 m with M^-1 = M^T diag(1/9, 1/36, 1/36, 1/6, 1/12, 1/6, 1/12,
// 1/4, 1/4)
template <class C>
__device__ __forceinline__ void from_moments(const C m[9], C f[9]) {
  C a0 = m[0] * C(1.0 / 9.0), a1 = m[1] * C(1.0 / 36.0),
    a2 = m[2] * C(1.0 / 36.0), a3 = m[3] * C(1.0 / 6.0),
    a4 = m[4] * C(1.0 / 12.0), a5 = m[5] * C(1.0 / 6.0),
    a6 = m[6] * C(1.0 / 12.0), a7 = m[7] * C(0.25), a8 = m[8] * C(0.25);
  C bax = a0 - a1 - C(2) * a2;   // axis directions
  C bdg = a0 + C(2) * a1 + a2;   // diagonal directions
  C px = a3 - C(2) * a4, py = a5 - C(2) * a6;
  C qx = a3 + a4, qy = a5 + a6;
  f[0] = a0 - C(4) * a1 + C(4) * a2;
  f[1] = bax + px + a7;
  f[3] = bax - px + a7;
  f[2] = bax + py - a7;
  f[4] = bax - py - a7;
  f[5] = bdg + qx + qy + a8;
  f[6] = bdg - qx + qy - a8;
  f[7] = bdg - qx - qy + a8;
  f[8] = bdg + qx - qy - a8;
}

}  // namespace lbpc
