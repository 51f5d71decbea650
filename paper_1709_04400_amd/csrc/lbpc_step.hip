// lbpc_step.hip -- the fused coupled time step for gfx950.
//
// One launch performs one whole time step (pull-streaming, moments, EOS,
// force, velocity, thermal source, both MRT collisions, store).  Layout and
// schedule:
//   * each buffer interleaves the rows of its nine direction arrays,
//     [ny][9][nx]; two buffers, ping-pong.  FP64 keeps f and g in buffers of
//     their own; the other forms store f and g of a direction as one pair
//     (8 bytes in FP32, a 32-bit word of two binary16 in the FP16 form, whose
//     rest populations are an FP32 pair per node).  The kernel reads
//     post-collision f*(t-1), g*(t-1) (or pre-collision f(t), g(t) right
//     after an initialisation: "fresh") and writes f*(t), g*(t);
//   * a block of BLOCK threads (64 to 512: one to eight wave64) owns a strip
//     of at most BLOCK - 4 columns plus 2 halo columns per side (one column
//     per thread) and a run of H rows, and marches along the rows (up or
//     down, alternating between vertically adjacent runs).  Iteration r:
//       A(r)   rho, j, T of row r from its pulled f, g; EOS (FP64): psi and
//              T (dp/dT)_rho -> LDS rings (5 rows) / registers
//       B(r-1) interaction force from psi rows r-2..r, buoyancy, velocity
//              -> LDS ring; flow MRT collision of row r-1, store f* (the
//              paired forms hold f* one iteration, to store it with g*)
//       pull of the next row(s) issued here, in flight during C2
//       C(r-2) isotropic differences of T, v (and rho) on rows r-3..r-1,
//              thermal source phi, S0, improved thermal MRT collision of
//              row r-2 (or a BGK collision: the Gong-Cheng model, or the
//              BGK form of the improved model), store g* (with f* in the
//              paired forms), phi
//     so every pulled value is loaded from memory once per block (halo
//     columns and the 4 warm-up rows aside) and the 2-hop stencil dependence
//     (div v needs v one node away, which needs psi two nodes away) never
//     goes to memory;
//   * pulled values wait as loaded (register images) until used: FP64 pulls
//     one row ahead and holds f one row and g two rows in registers; the
//     4- and 2-byte storage forms pull two rows ahead and keep cooked g of
//     the rows waiting for C in a per-thread LDS ring;
//   * a diagnostic launch (DIAG) also sums, in FP64, the fields of the time
//     level it starts from over the block's own nodes (at C, where rho, T
//     and v of the node are at hand) and reduces them across the wave
//     (butterfly shuffles), then across the block, into one record per
//     tile; a no-store diagnostic launch computes the same without storing
//     anything (the state stays as it is).
// Non-periodic sides: the pull applies bounce-back / open rules at edge
// nodes, and LDS reads of a ghost neighbour take the nearest lattice node's
// values with the ghost temperature / velocity rule.
#include <type_traits>

#include "lbpc_device.h"

namespace lbpc {

// Tile of this block.  Workgroups are dealt to the 8 XCDs round-robin; with
// xcd_order the tiles are renumbered so that the blocks one XCD runs at the
// same time are x-neighbours sharing halo columns in that XCD's L2.
__device__ __forceinline__ void block_tile(const StepParams& p, int& bx,
                                           int& by) {
  const int nb = p.nbx * p.nby;
  int b = blockIdx.x;
  if (p.xcd_order) {
    // XCD j runs blocks j, j+8, j+16, ...; the first `full` XCDs get
    // `per` tiles each, the others per - 1, in consecutive tile order
    const int per = (nb + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    const int full = nb - 8 * (per - 1);
    b = xcd < full ? xcd * per + k
                   : full * per + (xcd - full) * (per - 1) + k;
  }
  by = b / p.nbx;
  bx = b - by * p.nbx;
}

// waves per SIMD the register budget is sized for, and how many rows ahead
// the pull runs: 1 for FP64, 2 for the reduced-precision forms (their g
// queue sits in LDS, for which FP64 has no room).  FP64 holds its queues of
// pulled values in 64-bit registers, and the FP32 forms hold f* of a row as
// nine more registers until its (f, g) pairs are stored: both fit two waves
// per SIMD.  (At three, the FP32 forms spilled; storing each side of the
// pairs separately instead left partial writes that cost the walled
// 256-lattice batch 37 %.)  The FP16 forms' f and g share their loaded
// registers, which leaves room for three.
template <int P> struct StepOcc {
  static constexpr int waves = P >= 3 ? 3 : 2;
  static constexpr int prefetch = P == 0 ? 1 : 2;
};

// One tile: strip bx (W columns + halo), row run by (H rows), of the lattice
// described by p.
// Diagnostic record of a tile, 8 FP64 values: sum rho, sum T, sum rho T,
// liquid area, count above the mid density, sum S0, max |v|^2, non-finite.
constexpr int DIAG_VALS = 8;

// Side and hot-spot temperatures of the stencil ghosts, in the compute type.
// HOLD: read once into registers.  FP64 needs that: with the parameter loads
// inside the row loop its compiler turned "ghost ? load of T_side : stencil
// value" into one load through a selected pointer, which moved stencil values
// into scratch memory on every row (16 B written per node).  The FP32 forms
// read them in place, as written at their use: any other form of the same
// reads cost the FP16 form's boundary-capable kernel four more spilled
// registers and 21 % on a walled lattice.
template <class C, bool HOLD> struct SideTemps;
template <class C> struct SideTemps<C, true> {
  C t[4], th;
  __device__ explicit SideTemps(const StepParams& p) {
#pragma unroll
    for (int i = 0; i < 4; ++i) t[i] = C(p.T_bc[i]);
    th = C(p.T_hot);
  }
  __device__ C side(int i) const { return t[i]; }
  __device__ C hot() const { return th; }
};
template <class C> struct SideTemps<C, false> {
  __device__ explicit SideTemps(const StepParams&) {}
};

// PROBE: the same loads and stores in the same schedule with the
// arithmetic left out (each node stores the values it pulled, phi its
// history): the memory time of the step's access pattern.
// MRT: the lattice runs one of the MRT thermal models (improved or
// compromised), so the Gong-Cheng and BGK-form branches are compiled out;
// the FP16-deviation form, bound by instruction issue, takes this
// instantiation (3 % faster at 4096^2, 73 -> 32 spilled scalar registers).
template <int P, bool GEN, int BLOCK, bool DIAG, bool PROBE = false,
          bool MRT = false>
__device__ __forceinline__ void step_tile(const StepParams& p, int bx, int by,
                                          int slot, double* __restrict__ dpart,
                                          bool nostore) {
  using Tr = Prec<P>;
  using S = typename Tr::S;
  using C = typename Tr::C;

  __shared__ C s_rho[RING][BLOCK];
  __shared__ C s_T[RING][BLOCK];
  __shared__ C s_psi[RING][BLOCK];
  __shared__ C s_vx[RING][BLOCK];
  __shared__ C s_vy[RING][BLOCK];

  const int t = threadIdx.x;
  const int nx = p.nx, ny = p.ny;
  const long long N = p.N;
  const int X0 = bx * p.W, X1 = min(X0 + p.W, nx);
  // FP64 and the FP16 forms: the strips holding a non-periodic x side may run
  // shorter row runs (their edge waves do more work per row).  The FP32
  // forms keep one height (the host sets He = H for them): the select alone
  // cost their boundary-capable kernels up to 6 %.  (In the FP16 forms it
  // costs nothing, and the node-referenced form's kernel compiled with it
  // ran a walled 4096^2 lattice 4 % faster at equal heights.)
  int Hr = p.H;
  if constexpr (GEN && (P == 0 || P >= 3)) {
    if (!p.perx && (bx == 0 || bx == p.nbx - 1)) Hr = p.He;
  }
  const int Y0 = by * Hr, Y1 = min(Y0 + Hr, ny);
  const int c = X0 - HALO + t;  // unwrapped column of this thread

  const S* __restrict__ fin = static_cast<const S*>(p.fin);
  const S* __restrict__ gin = static_cast<const S*>(p.gin);
  S* __restrict__ fout = static_cast<S*>(p.fout);
  S* __restrict__ gout = static_cast<S*>(p.gout);
  const Gbl<C>* __restrict__ phiv = gbl(static_cast<const C*>(p.phi));
  Gbl<C>* __restrict__ phio = gbl(static_cast<C*>(p.phi_out));

  // column roles
  bool ghostc = false;
  int cw = c;
  if (c < 0 || c >= nx) {
    if (p.perx)
      cw = c < 0 ? c + nx : c - nx;
    else
      ghostc = true;
  }
  const bool doA = (c < X1 + HALO) && !ghostc;
  const bool doB = (c >= X0 - 1) && (c < X1 + 1) && !ghostc;
  const bool doC = (c >= X0) && (c < X1);
  // LDS column of the left / right neighbour (a clamped ghost reads the
  // nearest lattice column, which is this thread's own column)
  int ttm = t - 1, ttp = t + 1;
  if (GEN && !p.perx) {
    if (c - 1 < 0) ttm = t;
    if (c + 1 >= nx) ttp = t;
  }

  const Shift<P> sh(p);
  C sf[Q], sg[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    sf[a] = C(p.s_f[a]);
    sg[a] = C(p.s_g[a]);
  }

  // node-referenced FP16 form: the reference (binary16 rho or T, from the
  // ring `ring`) of each node that pulls one of the eight values node (x, y)
  // stores, x + e_a (s0, sU, sD: ring slots of rows y, y + 1, y - 1,
  // clamped like the stencil's), or the node's own where e_a leaves the
  // lattice across a wall (a value leaving across an open side is never
  // pulled); r[0] is the node's own.
  auto dest_ref = [&](const C (*ring)[BLOCK], int s0, int sU, int sD, int x,
                      int y, float r[Q]) __attribute__((always_inline)) {
    constexpr int ROW[Q] = {0, 0, 1, 0, 2, 1, 1, 2, 2};  // y, y+1, y-1
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const int sl = ROW[a] == 0 ? s0 : (ROW[a] == 1 ? sU : sD);
      const int tt = EXs[a] > 0 ? ttp : (EXs[a] < 0 ? ttm : t);
      r[a] = ref_round(ring[sl][tt]);
    }
    if (GEN) {
      const EdgeSides e(p, x, y, true);
      if (__builtin_amdgcn_ballot_w64(e.any()) != 0) {
#pragma unroll
        for (int a = 1; a < Q; ++a)
          if (e.wall(p, OPs[a])) r[a] = r[0];
      }
    }
  };

  // row r -> wrapped row, or -1 for a ghost row of a non-periodic y side
  auto wrap_row = [&](int r) -> int {
    if (r >= 0 && r < ny) return r;
    if (!p.pery) return -1;
    return r < 0 ? r + ny : r - ny;
  };

  // march direction alternates between vertically adjacent row runs, so the
  // rows two runs share are pulled by both at the same time (both at their
  // start or both at their end) and the second pull is served by L2
  const int dir = (by & 1) ? -1 : 1;
  const int nit = Y1 - Y0 + 4;
  const int rfirst = dir > 0 ? Y0 - 2 : Y1 + 1;
  const int rlast = rfirst + dir * (nit - 1);

  // Pulls are issued by every lane and every iteration, whether or not the
  // row is used: lanes without a node of their own read a clamped column,
  // rows past the run read its last row and ghost rows the nearest lattice
  // row (all recently read, so cache hits), and those values are never
  // used.  With no branch around the loads the compiler's wait counts
  // follow only the loads actually in flight.
  const int cl = cw < 0 ? 0 : (cw >= nx ? nx - 1 : cw);
  auto pull_row = [&](int rt, typename Tr::R* fr, typename Tr::R* gr) {
    const int rc = dir > 0 ? min(rt, rlast) : max(rt, rlast);
    int rw = wrap_row(rc);
    if (rw < 0) rw = rc < 0 ? 0 : ny - 1;
    pull_raw<P, GEN>(p, fin, gin, cl, rw, fr, gr);
  };

  // Pulled values stay as loaded (register images) until they are used, so
  // the loads of a row run while earlier rows are computed.
  //  PD = 1: row r is loaded one iteration ahead into slot 0 of F / G; f
  //    waits one more row in fq1 for the flow collision, g two rows in
  //    gq1, gq2 for the thermal collision.
  //  PD = 2: rows r+1 and r+2 are in flight in a 3-slot ring F / G (slot =
  //    iteration mod 3; the loop is unrolled by 3 so every slot is a set of
  //    registers and no in-flight load is ever moved); F keeps row r for
  //    the flow collision of the next iteration, and the thermal collision
  //    two rows later reads g of its row, as cooked at A, from a per-thread
  //    LDS ring.
  // Also carried: j (row r-1), T dp/dT (rows r-1, r-2) and 1/rho (row r-2)
  // of this thread's own column.
  constexpr int PD = StepOcc<P>::prefetch;
  constexpr int NS = PD == 1 ? 1 : 3;
  using R = typename Tr::R;
  R F[NS][Q], G[NS][Q], fq1[Q], gq1[Q], gq2[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
#pragma unroll
    for (int k = 0; k < NS; ++k) F[k][a] = G[k][a] = R(0);
    fq1[a] = gq1[a] = gq2[a] = R(0);
  }
  __shared__ C s_g[PD == 2 ? 3 : 1][PD == 2 ? Q : 1][PD == 2 ? BLOCK : 1];
  C jx1 = C(0), jy1 = C(0), tdp1 = C(0), tdp2 = C(0), irq = C(0);
  const SideTemps<C, GEN && P == 0> stemp(p);
  // paired forms: f and g of a direction share a word, and f* of a row is
  // ready one iteration before g* (C1 runs a row ahead of C2), so f* waits
  // here as its stored images (pack_f) until C2 stores the pairs
  unsigned int hf1[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) hf1[a] = 0u;
  // diagnostic sums of this thread's own nodes (DIAG only)
  double d_m = 0.0, d_T = 0.0, d_e = 0.0, d_a = 0.0, d_c = 0.0, d_s = 0.0,
         d_v = 0.0, d_bad = 0.0;
  const bool skip = DIAG && nostore;

#pragma unroll
  for (int k = 0; k < PD; ++k) pull_row(rfirst + k * dir, F[k], G[k]);

  // one iteration; kc is the ring slot of row r (always 0 for PD = 1)
  auto iteration = [&](auto kc, const int it) __attribute__((always_inline)) {
    constexpr int k = decltype(kc)::value;
    constexpr int kp = PD == 1 ? 0 : (k + 2) % 3;  // row r-1, then row r+2
    constexpr int k2 = PD == 1 ? 0 : (k + 1) % 3;  // g ring: row r-2
    const int r = rfirst + dir * it;
    const int sl0 = it % RING;                // slot of row r
    const int sl1 = (it + RING - 1) % RING;   // row r - dir
    const int sl2 = (it + RING - 2) % RING;   // row r - 2 dir
    const int sl3 = (it + RING - 3) % RING;   // row r - 3 dir
    unsigned int hfn[Q];  // f* of row r - dir (paired forms)
#pragma unroll
    for (int a = 0; a < Q; ++a) hfn[a] = hf1[a];

    // ------------------------------------------------------------ A(r)
    C jxn = C(0), jyn = C(0), tdpn = C(0);
    const int rwA = wrap_row(r);
    if (doA && rwA >= 0) {
      C fa[Q], ga[Q];
      cook_f<P, GEN>(p, sh, cw, rwA, F[k], G[k], fa);
      cook_g<P, GEN>(p, sh, cw, rwA, F[k], G[k], ga);
      if constexpr (PD == 2) {
#pragma unroll
        for (int a = 0; a < Q; ++a) s_g[k][a][t] = ga[a];
      }
      if constexpr (!PROBE) {
      const C sa = fa[1] + fa[2] + fa[3] + fa[4];
      const C sd = fa[5] + fa[6] + fa[7] + fa[8];
      const C rho = fa[0] + sa + sd;
      jxn = (fa[1] - fa[3]) + (fa[5] - fa[6] - fa[7] + fa[8]);
      jyn = (fa[2] - fa[4]) + (fa[5] + fa[6] - fa[7] - fa[8]);
      const C T = ga[0] + (ga[1] + ga[2] + ga[3] + ga[4]) +
                  (ga[5] + ga[6] + ga[7] + ga[8]);
      // Peng-Robinson EOS, Eq. (56), in FP64 with one reciprocal:
      //   p = (rho R T D2 - a th rho^2 D1) / (D1 D2),
      //   T dp/dT = (rho R T D2 + a kappa s sqrt(T/Tc) rho^2 D1) / (D1 D2),
      // D1 = 1 - b rho, D2 = 1 + 2 b rho - b^2 rho^2, s = 1 + kappa (1 -
      // sqrt(T/Tc)), th = s^2 (using T dth/dT = -kappa s sqrt(T/Tc))
      // the state a node may hold: psi^2 >= 0, 0 < rho < 1/b, finite T
      double psi;
      bool valid;
      if constexpr (sizeof(C) == 8) {
        const double rd = rho, Td = T;
        const double sq = sqrt(Td * p.inv_Tc);
        const double s = 1.0 + p.kappa * (1.0 - sq);
        const double brho = p.b * rd;
        const double D1 = 1.0 - brho, D2 = 1.0 + brho * (2.0 - brho);
        const double inv = 1.0 / (D1 * D2);
        const double rRT = rd * p.R * Td * D2;
        const double ar2 = p.a * rd * rd * D1;
        const double pe = (rRT - ar2 * s * s) * inv;
        const double psi2 = p.two_over_G * (pe - rd * (1.0 / 3.0));
        psi = sqrt(psi2 > 0.0 ? psi2 : 0.0);
        tdpn = C((rRT + ar2 * p.kappa * s * sq) * inv);
        valid = psi2 >= 0.0 && rd > 0.0 && brho < 1.0 && Td - Td == 0.0;
      } else {
        // FP32 arithmetic: the smooth factors (sqrt(T/Tc), s, 1/(D1 D2))
        // in FP32, the cancelling combinations (repulsive - attractive
        // pressure, then p - rho c_s^2) in FP64
        const float sq = fsqrt(T * float(p.inv_Tc));
        const float s = 1.0f + float(p.kappa) * (1.0f - sq);
        const float brho = float(p.b) * rho;
        const float D1 = 1.0f - brho, D2 = 1.0f + brho * (2.0f - brho);
        const float inv = recip(D1 * D2);
        const double rd = rho;
        const double rRT = rd * p.R * (double)T * (double)D2;
        const double ar2 = p.a * rd * rd * (double)D1;
        const double th = (double)s * (double)s;
        const double pe = (rRT - ar2 * th) * (double)inv;
        const double psi2 = p.two_over_G * (pe - rd * (1.0 / 3.0));
        psi = fsqrt(float(psi2 > 0.0 ? psi2 : 0.0));
        tdpn = C((rRT + ar2 * (p.kappa * (double)(s * sq))) * (double)inv);
        valid = psi2 >= 0.0 && rd > 0.0 && rd * p.b < 1.0 && T - T == 0.0f;
      }
      if (!valid) *p.bad = 1;
      s_rho[sl0][t] = rho;
      s_T[sl0][t] = T;
      s_psi[sl0][t] = C(psi);
      }  // !PROBE
    }
    __syncthreads();

    // ------------------------------------------------ B(r-1) and C1(r-1)
    C irn = C(0);
    if constexpr (PROBE) {
      const int rb = r - dir;
      if (doC && rb >= Y0 && rb < Y1) {
        C fo[Q];
        cook_f<P, GEN>(p, sh, c, rb, PD == 1 ? fq1 : F[kp],
                       PD == 1 ? fq1 : G[kp], fo);
#pragma unroll
        for (int a = 0; a < Q; ++a) fo[a] -= sh.f(a);
        if constexpr (P == 4) {
          const float z[Q] = {};  // (stored values unused)
          pack_f_local(fo, z, hfn);
        } else if constexpr (Tr::paired) {
          pack_f<P>(fo, hfn);
        } else {
          store_node<P>(fout, nx, rb, c, fo);
        }
      }
    } else {
      const int rb = r - dir;
      const bool ghostr = (rb < 0 || rb >= ny) && !p.pery;
      if (doB && !ghostr && rb >= Y0 - 1 && rb <= Y1) {
        // psi rows rb-1, rb, rb+1 (clamped at non-periodic y sides)
        int sm = dir > 0 ? sl2 : sl0, sp = dir > 0 ? sl0 : sl2;
        if (GEN && !p.pery) {
          if (rb - 1 < 0) sm = sl1;
          if (rb + 1 >= ny) sp = sl1;
        }
        const C pc = s_psi[sl1][t];
        C pE = s_psi[sl1][ttp], pW = s_psi[sl1][ttm];
        C pN = s_psi[sp][t], pS = s_psi[sm][t];
        C pNE = s_psi[sp][ttp], pNW = s_psi[sp][ttm];
        C pSE = s_psi[sm][ttp], pSW = s_psi[sm][ttm];
        if (GEN && p.wet) {
          // a neighbour across a wall (either crossed side, at corners)
          // takes psi of its nearest node's virtual density; the clamped
          // ring slot and column above are that node
          const bool c0 = !p.perx && c - 1 < 0, c1 = !p.perx && c + 1 >= nx;
          const bool r0 = !p.pery && rb - 1 < 0, r1 = !p.pery && rb + 1 >= ny;
          if (__builtin_amdgcn_ballot_w64(c0 || c1 || r0 || r1) != 0) {
            const bool w0 = c0 && p.bc[0] == BC_WALL;
            const bool w1 = c1 && p.bc[1] == BC_WALL;
            const bool w2 = r0 && p.bc[2] == BC_WALL;
            const bool w3 = r1 && p.bc[3] == BC_WALL;
            auto wp = [&](int sl, int tt) {
              return C(wall_psi(p, double(s_rho[sl][tt]), double(s_T[sl][tt])));
            };
            if (w1) pE = wp(sl1, ttp);
            if (w0) pW = wp(sl1, ttm);
            if (w3) pN = wp(sp, t);
            if (w2) pS = wp(sm, t);
            if (w1 || w3) pNE = wp(sp, ttp);
            if (w0 || w3) pNW = wp(sp, ttm);
            if (w1 || w2) pSE = wp(sm, ttp);
            if (w0 || w2) pSW = wp(sm, ttm);
          }
        }
        // F_m = -G psi sum_a w_a psi(x+e_a) e_a = -G psi (sx, sy)
        const C sx = C(1.0 / 3.0) * (pE - pW) +
                     C(1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
        const C sy = C(1.0 / 3.0) * (pN - pS) +
                     C(1.0 / 12.0) * ((pNE - pSE) + (pNW - pSW));
        const C mGpc = C(-p.G) * pc;
        const C Fmx = mGpc * sx, Fmy = mGpc * sy;
        const C rho = s_rho[sl1][t];
        const C drho = rho - C(p.rho_ave);
        const C Fx = Fmx + drho * C(p.gx), Fy = Fmy + drho * C(p.gy);
        irn = recip(rho);
        const C vx = (jx1 + C(0.5) * Fx) * irn;
        const C vy = (jy1 + C(0.5) * Fy) * irn;
        s_vx[sl1][t] = vx;
        s_vy[sl1][t] = vy;

        if (doC && rb >= Y0 && rb < Y1 && !skip) {
          // flow MRT collision with the forcing scheme of the flow model;
          // |F_m|^2 / psi^2 = G^2 (sx^2 + sy^2), folded into sig1, sig2
          C m[Q], ms[Q], fo[Q], fb[Q];
          cook_f<P, GEN>(p, sh, c, rb, PD == 1 ? fq1 : F[kp],
                         PD == 1 ? fq1 : G[kp], fb);
          to_moments(fb, m);
          const C v2 = vx * vx + vy * vy;
          C meq[Q];
          meq[0] = rho;
          meq[1] = rho * (C(-2) + C(3) * v2);
          meq[2] = rho * (C(1) - C(3) * v2);
          meq[3] = rho * vx;
          meq[4] = -rho * vx;
          meq[5] = rho * vy;
          meq[6] = -rho * vy;
          meq[7] = rho * (vx * vx - vy * vy);
          meq[8] = rho * vx * vy;
          const C vF = vx * Fx + vy * Fy;
          const C s2 = sx * sx + sy * sy;
          C Sf[Q];
          Sf[0] = C(0);
          Sf[1] = C(6) * vF + C(p.sig1) * s2;
          Sf[2] = -C(6) * vF - C(p.sig2) * s2;
          Sf[3] = Fx;
          Sf[4] = -Fx;
          Sf[5] = Fy;
          Sf[6] = -Fy;
          Sf[7] = C(2) * (vx * Fx - vy * Fy);
          Sf[8] = vx * Fy + vy * Fx;
#pragma unroll
          for (int k = 0; k < Q; ++k)
            ms[k] = m[k] - sf[k] * (m[k] - meq[k]) +
                    (C(1) - C(0.5) * sf[k]) * Sf[k];
          from_moments(ms, fo);
#pragma unroll
          for (int a = 0; a < Q; ++a) fo[a] -= sh.f(a);
          if constexpr (P == 4) {
            float rr[Q];
            dest_ref(s_rho, sl1, sp, sm, c, rb, rr);
            pack_f_local(fo, rr, hfn);
          } else if constexpr (Tr::paired) {
            pack_f<P>(fo, hfn);
          } else {
            store_node<P>(fout, nx, rb, c, fo);
          }
        }
      }
    }
    // history of the row C2 updates below (phi(t-1), and T v(t-1) of the
    // BGK form), loaded before the row prefetch: loads complete in order,
    // so waiting for a load issued after the prefetch would wait for the
    // whole prefetch as well
    C hphi = C(0), htx = C(0), hty = C(0);
    {
      const int yc = r - 2 * dir;
      if (doC && yc >= Y0 && yc < Y1 && p.phi_valid &&
          (p.improved || (!MRT && p.bgk))) {
        const long long o = (long long)yc * nx + c;
        hphi = phiv[o];
        if ((!MRT && p.bgk)) {
          htx = phiv[N + o];
          hty = phiv[2 * N + o];
        }
      }
    }
    R gn[Q];
    if constexpr (PD == 1) {
      // f of row r waits one row for its collision; row r + dir is pulled
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        fq1[a] = F[0][a];
        gn[a] = R(0);
      }
      pull_row(r + dir, F[0], gn);
    } else {
      // row r + 2 dir into the slot row r - 1 has just left
      pull_row(r + 2 * dir, F[kp], G[kp]);
    }
    __syncthreads();

    // -------------------------------------------------------------- C2(r-2)
    if constexpr (PROBE) {
      const int yc = r - 2 * dir;
      if (doC && yc >= Y0 && yc < Y1) {
        C go[Q];
        if constexpr (PD == 1) {
          cook_g<P, GEN>(p, sh, c, yc, gq2, gq2, go);
        } else {
#pragma unroll
          for (int a = 0; a < Q; ++a) go[a] = s_g[k2][a][t];
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) go[a] -= sh.g(a);
        phio[(long long)yc * nx + c] = hphi;
        if constexpr (P == 4) {
          const float z[Q] = {};
          store_pairs_local(p, fout, p.rout, nx, yc, c, hf1, go, z, 0u);
        } else if constexpr (Tr::paired) {
          store_pairs<P>(fout, p.rout, nx, yc, c, hf1, go);
        } else {
          store_node<P>(gout, nx, yc, c, go);
        }
      }
    } else {
      const int yc = r - 2 * dir;
      const int slN = dir > 0 ? sl1 : sl3, slS = dir > 0 ? sl3 : sl1;
      if (doC && yc >= Y0 && yc < Y1) {
        const C T = s_T[sl2][t];
        const C vx = s_vx[sl2][t], vy = s_vy[sl2][t];
        // neighbour values (E, W, N, S, NE, NW, SE, SW); a ghost neighbour
        // across a non-periodic side reads the nearest lattice node (the
        // LDS column and ring row are clamped), then takes the side
        // temperature and, across a wall, zero velocity
        C Tn[8], vxn[8], vyn[8], rn[8];
        constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
        constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
        const bool r2 = GEN && !p.pery && yc == 0;
        const bool r3 = GEN && !p.pery && yc == ny - 1;
        const int sN = r3 ? sl2 : slN, sS = r2 ? sl2 : slS;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
          const int tt = DX[k] > 0 ? ttp : (DX[k] < 0 ? ttm : t);
          const int sl = DY[k] > 0 ? sN : (DY[k] < 0 ? sS : sl2);
          Tn[k] = s_T[sl][tt];
          vxn[k] = s_vx[sl][tt];
          vyn[k] = s_vy[sl][tt];
          rn[k] = p.lambda_mode ? s_rho[sl][tt] : C(0);
        }
        if (GEN) {
          const bool c0 = !p.perx && c == 0, c1 = !p.perx && c == nx - 1;
          const bool edge =
              __builtin_amdgcn_ballot_w64(c0 || c1 || r2 || r3) != 0;
          // FP32 arithmetic: a row away from the y sides (r2, r3 are
          // wave-uniform) takes only the x-side ghosts, which take that
          // side's temperature and, across a wall, zero velocity.  Not FP64,
          // whose boundary-capable kernel is at its register cap and ran
          // 1.9 % slower with it.
          bool xonly = false;
          if constexpr (sizeof(C) == 4) xonly = !(r2 || r3);
          if (edge && xonly) {
            const bool w0 = p.bc[0] == BC_WALL, w1 = p.bc[1] == BC_WALL;
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              if (DX[k] == 0) continue;
              const bool ox = DX[k] > 0 ? c1 : c0;
              const bool wall = ox && (DX[k] > 0 ? w1 : w0);
              Tn[k] = ox ? C(p.T_bc[DX[k] > 0 ? 1 : 0]) : Tn[k];
              vxn[k] = wall ? C(0) : vxn[k];
              vyn[k] = wall ? C(0) : vyn[k];
            }
          } else if (edge) {
#pragma unroll
            for (int k = 0; k < 8; ++k) {
              const int xs = DX[k] > 0 ? 1 : 0, ys = DY[k] > 0 ? 3 : 2;
              const bool ox = DX[k] > 0 ? c1 : (DX[k] < 0 ? c0 : false);
              const bool oy = DY[k] > 0 ? r3 : (DY[k] < 0 ? r2 : false);
              const bool wall = (ox && p.bc[xs] == BC_WALL) ||
                                (oy && p.bc[ys] == BC_WALL);
              int col = c + DX[k];
              if (ox) col = c;
              else if (col < 0) col += nx;
              else if (col >= nx) col -= nx;
              C Tg;
              if constexpr (P == 0 && GEN) {
                const C Ty = ys == 2 ? (col >= p.hot_x0 && col < p.hot_x1
                                            ? stemp.hot()
                                            : stemp.side(2))
                                     : stemp.side(3);
                Tg = oy ? Ty : stemp.side(xs);
              } else {
                const C Ty = ys == 2 ? (col >= p.hot_x0 && col < p.hot_x1
                                            ? C(p.T_hot)
                                            : C(p.T_bc[2]))
                                     : C(p.T_bc[3]);
                Tg = oy ? Ty : C(p.T_bc[xs]);
              }
              Tn[k] = (ox || oy) ? Tg : Tn[k];
              vxn[k] = wall ? C(0) : vxn[k];
              vyn[k] = wall ? C(0) : vyn[k];
            }
          }
        }
        // isotropic differences: d_i X = 3 sum_a w_a X(x+e_a) e_ai,
        // lap X = 6 sum_a w_a (X(x+e_a) - X(x))
        const C third = C(1.0 / 3.0), twelfth = C(1.0 / 12.0);
        const C dTx = third * (Tn[0] - Tn[1]) +
                      twelfth * ((Tn[4] - Tn[5]) + (Tn[6] - Tn[7]));
        const C dTy = third * (Tn[2] - Tn[3]) +
                      twelfth * ((Tn[4] - Tn[6]) + (Tn[5] - Tn[7]));
        const C lapT =
            C(2.0 / 3.0) * ((Tn[0] + Tn[1]) + (Tn[2] + Tn[3]) - C(4) * T) +
            C(1.0 / 6.0) * ((Tn[4] + Tn[5]) + (Tn[6] + Tn[7]) - C(4) * T);
        const C divv = third * (vxn[0] - vxn[1]) +
                       twelfth * ((vxn[4] - vxn[5]) + (vxn[6] - vxn[7])) +
                       third * (vyn[2] - vyn[3]) +
                       twelfth * ((vyn[4] - vyn[6]) + (vyn[5] - vyn[7]));
        // phi of Eq. (28): div(lambda grad T)/(rho c_V) - k lap T
        //                  + (T - T (dp/dT)/(rho c_V)) div v
        C phi;
        if ((!MRT && p.gc)) {
          // Eq. (13): T (1 - (dp/dT)/(rho c_V)) div v
          phi = (T - tdp2 * irq * C(p.inv_cv)) * divv;
        } else {
          C lam_term;
          if (p.lambda_mode == 0) {
            lam_term = C(p.lam_over_cv) * irq * lapT;
          } else {
            // lambda = rho c_V chi: chi (lap T + grad rho . grad T / rho)
            const C drx = third * (rn[0] - rn[1]) +
                          twelfth * ((rn[4] - rn[5]) + (rn[6] - rn[7]));
            const C dry = third * (rn[2] - rn[3]) +
                          twelfth * ((rn[4] - rn[6]) + (rn[5] - rn[7]));
            lam_term = C(p.chi) * (lapT + irq * (drx * dTx + dry * dTy));
          }
          phi = lam_term - C(p.k_th) * lapT +
                (T - tdp2 * irq * C(p.inv_cv)) * divv;
        }
        const long long o = (long long)yc * nx + c;
        C S0 = phi;
        if (p.improved || (!MRT && p.bgk)) {
          const C prev = p.phi_valid ? hphi : phi;
          S0 = phi + C(0.5) * (phi - prev);
        }
        if constexpr (DIAG) {
          // FP64 sums of the time level this step starts from
          const double rd = double(s_rho[sl2][t]);
          const double Td = double(T), vxd = double(vx), vyd = double(vy);
          d_m += rd;
          d_T += Td;
          d_e += rd * Td;
          double fr = (rd - p.rho_v) / (p.rho_l - p.rho_v);
          fr = fr < 0.0 ? 0.0 : (fr > 1.0 ? 1.0 : fr);
          d_a += fr;
          d_c += rd > 0.5 * (p.rho_l + p.rho_v) ? 1.0 : 0.0;
          d_s += double(S0);
          const double sp = vxd * vxd + vyd * vyd;
          d_v = sp > d_v ? sp : d_v;
          if (!(rd - rd == 0.0 && Td - Td == 0.0 && sp - sp == 0.0))
            d_bad = 1.0;
        }
        if (!skip) {
        phio[o] = phi;
        C go[Q], gb[Q];
        if constexpr (PD == 1) {
          cook_g<P, GEN>(p, sh, c, yc, gq2, gq2, gb);
        } else {
#pragma unroll
          for (int a = 0; a < Q; ++a) gb[a] = s_g[k2][a][t];
        }
        if ((!MRT && p.gc) || (!MRT && p.bgk)) {
          // BGK collisions.  Gong-Cheng, Eq. (12): g^eq of Eq. (14), source
          // omega_a phi, tau_g = lambda/(rho c_V c_s^2) + 1/2.  BGK form of
          // the improved model, Eq. (33): g^eq of Eq. (29), source
          // omega_a S0 (Eq. 32) and the correction of Eq. (31) with
          // d_t(T v) = T v(t) - T v(t-1) (history after phi in the array)
          C itau, base, q2, src, cf = C(0), dx = C(0), dy = C(0);
          if ((!MRT && p.gc)) {
            itau = recip(C(p.gc_ta) * irq + C(p.gc_tb));
            base = C(1) - C(1.5) * (vx * vx + vy * vy);
            q2 = C(4.5);
            src = phi;
          } else {
            itau = C(p.bgk_itau);
            base = C(1);
            q2 = C(0);
            src = S0;
            cf = C(p.bgk_cfac);
            const C tvx = T * vx, tvy = T * vy;
            if (p.phi_valid) {
              dx = tvx - htx;
              dy = tvy - hty;
            }
            phio[N + o] = tvx;
            phio[2 * N + o] = tvy;
          }
#pragma unroll
          for (int a = 0; a < Q; ++a) {
            const C eu = C(EXs[a]) * vx + C(EYs[a]) * vy;
            const C wa = C(w_lat(a));
            const C geq = wa * T * (base + eu * (C(3) + q2 * eu));
            go[a] = gb[a] - (gb[a] - geq) * itau + wa * src +
                    cf * wa * (C(EXs[a]) * dx + C(EYs[a]) * dy);
          }
        } else {
          // improved thermal MRT collision: Eqs. (45), (46), (53)-(55)
          C n[Q], ns[Q];
          to_moments(gb, n);
          const C neq4 = -T * vx, neq6 = -T * vy;
          ns[0] = T + S0;
          ns[1] = n[1] - sg[1] * (n[1] + C(2) * T);
          ns[2] = n[2] - sg[2] * (n[2] - C(2) * T);
          ns[3] = n[3] - sg[3] * (n[3] - T * vx);
          ns[4] = n[4] - sg[4] * (n[4] - neq4);
          ns[5] = n[5] - sg[5] * (n[5] - T * vy);
          ns[6] = n[6] - sg[6] * (n[6] - neq6);
          ns[7] = n[7] - sg[7] * n[7];
          ns[8] = n[8] - sg[8] * n[8];
          if (p.improved) {
            ns[3] += (C(1) - C(0.5) * sg[3]) * sg[4] * (n[4] - neq4);
            ns[5] += (C(1) - C(0.5) * sg[5]) * sg[6] * (n[6] - neq6);
          }
          from_moments(ns, go);
        }
#pragma unroll
        for (int a = 0; a < Q; ++a) go[a] -= sh.g(a);
        if constexpr (P == 4) {
          float tr[Q];
          dest_ref(s_T, sl2, sN, sS, c, yc, tr);
          store_pairs_local(p, fout, p.rout, nx, yc, c, hf1, go, tr,
                            ref_word(s_rho[sl2][t], T));
        } else if constexpr (Tr::paired) {
          store_pairs<P>(fout, p.rout, nx, yc, c, hf1, go);
        } else {
          store_node<P>(gout, nx, yc, c, go);
        }
        }  // !skip
      }
    }

    if constexpr (PD == 1) {
      // rotate the per-column g queue
#pragma unroll
      for (int a = 0; a < Q; ++a) {
        gq2[a] = gq1[a];
        gq1[a] = G[0][a];
        G[0][a] = gn[a];
      }
    }
    jx1 = jxn;
    jy1 = jyn;
    tdp2 = tdp1;
    tdp1 = tdpn;
    irq = irn;
#pragma unroll
    for (int a = 0; a < Q; ++a) hf1[a] = hfn[a];
  };

  if constexpr (PD == 1) {
    for (int it = 0; it < nit; ++it)
      iteration(std::integral_constant<int, 0>{}, it);
  } else {
    // whole groups of three: iterations past nit issue no loads and their
    // rows fall outside the B / C ranges, so they only cost arithmetic;
    // without guards every path into a group has the same loads in flight,
    // which keeps the compiler's wait counts exact
    for (int it = 0; it < nit; it += 3) {
      iteration(std::integral_constant<int, 0>{}, it);
      iteration(std::integral_constant<int, 1>{}, it + 1);
      iteration(std::integral_constant<int, 2>{}, it + 2);
    }
  }

  if constexpr (DIAG) {
    // butterfly over the wave (every lane ends with the wave's total; lane 0
    // keeps it), then the waves in order: a fixed order, so the record is
    // the same on every run
    __shared__ double s_red[BLOCK / 64][DIAG_VALS];
    double v[DIAG_VALS] = {d_m, d_T, d_e, d_a, d_c, d_s, d_v, d_bad};
#pragma unroll
    for (int k = 0; k < DIAG_VALS; ++k) {
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(v[k], off, 64);
        v[k] = k >= 6 ? (o > v[k] ? o : v[k]) : v[k] + o;
      }
    }
    if ((t & 63) == 0) {
#pragma unroll
      for (int k = 0; k < DIAG_VALS; ++k) s_red[t >> 6][k] = v[k];
    }
    __syncthreads();
    if (t < DIAG_VALS) {
      double acc = s_red[0][t];
#pragma unroll
      for (int w = 1; w < BLOCK / 64; ++w) {
        const double o = s_red[w][t];
        acc = t >= 6 ? (o > acc ? o : acc) : acc + o;
      }
      dpart[(long long)slot * DIAG_VALS + t] = acc;
    }
  }
}

// Waves per SIMD a block shape can reach: a 512-thread block (8 waves) with
// its 100-104 KiB of LDS runs one per CU, i.e. 2 waves per SIMD, whatever
// the form's register budget would allow.
template <int P, int BLOCK> struct BlockOcc {
  static constexpr int waves = BLOCK == 512 ? 2 : StepOcc<P>::waves;
};

template <int P, bool GEN, int BLOCK, bool DIAG, bool MRT = false>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    BlockOcc<P, BLOCK>::waves, BlockOcc<P, BLOCK>::waves))) void
k_step(StepParams p, double* dpart, int nostore) {
  int bx, by;
  block_tile(p, bx, by);
  step_tile<P, GEN, BLOCK, DIAG, false, MRT>(p, bx, by, by * p.nbx + bx,
                                             dpart, nostore != 0);
}

// The memory schedule of k_step without its arithmetic (see step_tile):
// reads the state and the phi history, writes the other buffer and
// phi_out (the host points phi_out at scratch).
template <int P, int BLOCK>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    BlockOcc<P, BLOCK>::waves, BlockOcc<P, BLOCK>::waves))) void
k_step_probe(StepParams p) {
  int bx, by;
  block_tile(p, bx, by);
  step_tile<P, false, BLOCK, false, true>(p, bx, by, 0, nullptr, false);
}

hipError_t launch_step_probe(const StepParams& p, int prec, hipStream_t s) {
  const dim3 grid(p.nbx * p.nby);
  if (!(p.perx && p.pery)) return hipErrorInvalidValue;
#define LBPC_PROBE_BW(PR)                                                    \
  if (p.bw == 512)                                                           \
    hipLaunchKernelGGL((k_step_probe<PR, 512>), grid, dim3(512), 0, s, p);   \
  else                                                                       \
    hipLaunchKernelGGL((k_step_probe<PR, 256>), grid, dim3(256), 0, s, p);
  switch (prec) {
    case 0: LBPC_PROBE_BW(0); break;
    case 1: LBPC_PROBE_BW(1); break;
    case 2: LBPC_PROBE_BW(2); break;
    case 3: LBPC_PROBE_BW(3); break;
    case 4: LBPC_PROBE_BW(4); break;
    default: return hipErrorInvalidValue;
  }
#undef LBPC_PROBE_BW
  return hipGetLastError();
}

// Batched form: many independent lattices, one persistent launch per step.
// `table` holds each case's parameters for both buffer parities; `work`
// lists (case, bx, by, slot) tiles, costliest first (slot: the tile's
// diagnostic record; the records of one lattice are contiguous); every
// block walks the list with a stride of the grid size, so each tile is done
// exactly once and every block leaves when the list ends.
struct WorkItem {
  int c, bx, by, slot;
};

template <int P, int BLOCK, bool GEN, bool DIAG>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(
    BlockOcc<P, BLOCK>::waves, BlockOcc<P, BLOCK>::waves))) void
k_step_batch(const StepParams* __restrict__ table,
             const WorkItem* __restrict__ work, int nwork, int parity,
             double* dpart, int nostore) {
  for (int w = blockIdx.x; w < nwork; w += gridDim.x) {
    const WorkItem it = work[w];
    const StepParams& p = table[2 * it.c + parity];
    step_tile<P, GEN, BLOCK, DIAG>(p, it.bx, it.by, it.slot, dpart,
                                   nostore != 0);
    __syncthreads();  // the LDS rings are reused by the next tile
  }
}

// host-side launchers: one instantiation per storage precision, block
// width, boundary mode (GEN = some side is not periodic) and diagnostic mode
// (dpart != nullptr: sum the diagnostics into dpart; nostore: store nothing)
hipError_t launch_step(const StepParams& p, int prec, hipStream_t s,
                       double* dpart, int nostore) {
  const dim3 grid(p.nbx * p.nby);
  const bool gen = !(p.perx && p.pery);
  // lattices with a non-periodic side run the tile-list kernel
  if (gen) return hipErrorInvalidValue;
#define LBPC_LAUNCH_BW(PR, BW, M)                                              \
  if (dpart)                                                                   \
    hipLaunchKernelGGL((k_step<PR, false, BW, true, M>), grid, dim3(BW), 0, s, \
                       p, dpart, nostore);                                     \
  else                                                                         \
    hipLaunchKernelGGL((k_step<PR, false, BW, false, M>), grid, dim3(BW), 0,   \
                       s, p, dpart, 0);
#define LBPC_LAUNCH(PR, M)                                                     \
  if (p.bw == 64) {                                                            \
    LBPC_LAUNCH_BW(PR, 64, M)                                                  \
  } else if (p.bw == 128) {                                                    \
    LBPC_LAUNCH_BW(PR, 128, M)                                                 \
  } else if (p.bw == 512) {                                                    \
    LBPC_LAUNCH_BW(PR, 512, M)                                                 \
  } else {                                                                     \
    LBPC_LAUNCH_BW(PR, 256, M)                                                 \
  }
  switch (prec) {
    case 0: LBPC_LAUNCH(0, false); break;
    case 1: LBPC_LAUNCH(1, false); break;
    case 2: LBPC_LAUNCH(2, false); break;
    case 3:
      // the FP16 forms under an MRT thermal model take the instantiation
      // without the Gong-Cheng and BGK-form branches
      if (!p.gc && !p.bgk) {
        LBPC_LAUNCH(3, true);
      } else {
        LBPC_LAUNCH(3, false);
      }
      break;
    case 4:
      if (!p.gc && !p.bgk) {
        LBPC_LAUNCH(4, true);
      } else {
        LBPC_LAUNCH(4, false);
      }
      break;
    default: return hipErrorInvalidValue;
  }
#undef LBPC_LAUNCH
#undef LBPC_LAUNCH_BW
  return hipGetLastError();
}

hipError_t launch_step_batch(const StepParams* table, const void* work,
                             int nwork, int parity, int grid, int prec,
                             int bw, hipStream_t s, bool gen, double* dpart,
                             int nostore) {
  const WorkItem* wk = static_cast<const WorkItem*>(work);
#define LBPC_BL(PR, BW, G, D)                                                \
  hipLaunchKernelGGL((k_step_batch<PR, BW, G, D>), dim3(grid), dim3(BW), 0, \
                     s, table, wk, nwork, parity, dpart, nostore);
#define LBPC_BLAUNCH_BW(PR, BW)                                              \
  if (gen) {                                                                 \
    if (dpart) {                                                             \
      LBPC_BL(PR, BW, true, true)                                            \
    } else {                                                                 \
      LBPC_BL(PR, BW, true, false)                                           \
    }                                                                        \
  } else {                                                                   \
    if (dpart) {                                                             \
      LBPC_BL(PR, BW, false, true)                                           \
    } else {                                                                 \
      LBPC_BL(PR, BW, false, false)                                          \
    }                                                                        \
  }
#define LBPC_BLAUNCH(PR)                                                      \
  if (bw == 64) {                                                             \
    LBPC_BLAUNCH_BW(PR, 64)                                                   \
  } else if (bw == 128) {                                                     \
    LBPC_BLAUNCH_BW(PR, 128)                                                  \
  } else if (bw == 512) {                                                     \
    LBPC_BLAUNCH_BW(PR, 512)                                                  \
  } else {                                                                    \
    LBPC_BLAUNCH_BW(PR, 256)                                                  \
  }
  switch (prec) {
    case 0: LBPC_BLAUNCH(0); break;
    case 1: LBPC_BLAUNCH(1); break;
    case 2: LBPC_BLAUNCH(2); break;
    case 3: LBPC_BLAUNCH(3); break;
    case 4: LBPC_BLAUNCH(4); break;
    default: return hipErrorInvalidValue;
  }
#undef LBPC_BLAUNCH
#undef LBPC_BLAUNCH_BW
#undef LBPC_BL
  return hipGetLastError();
}

int work_item_bytes() { return (int)sizeof(WorkItem); }

}  // namespace lbpc
