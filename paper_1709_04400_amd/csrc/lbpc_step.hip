// lbpc_step.hip -- the fused coupled time step for gfx950.
//
// One launch performs one whole time step (pull-streaming, moments, EOS,
// force, velocity, thermal source, both MRT collisions, store).  Layout and
// schedule:
//   * distributions are SoA [9][ny][nx] per buffer, ping-pong; the kernel
//     reads post-collision f*(t-1), g*(t-1) (or pre-collision f(t), g(t)
//     right after an initialisation: "fresh") and writes f*(t), g*(t);
//   * a block of 256 threads (4 wave64) owns a strip of W = 252 columns plus
//     2 halo columns per side (one column per thread) and a run of H rows;
//     it marches up the rows.  Iteration r:
//       A(r)   pull f, g at row r; rho, j, T, psi -> LDS ring (5 rows)
//       B(r-1) interaction force from psi rows r-2..r, buoyancy, velocity
//              -> LDS ring; flow MRT collision of row r-1, store f*
//       C(r-2) isotropic differences of T, v (and rho) on rows r-3..r-1,
//              thermal source phi, S0, improved thermal MRT collision of
//              row r-2, store g*, phi
//     so every pulled value is loaded from memory exactly once per block
//     (halo columns aside) and the 2-hop stencil dependence (div v needs v
//     one node away, which needs psi two nodes away) never goes to memory;
//   * pulled f is held in registers for one row, pulled g for two.
// Non-periodic sides: the pull applies bounce-back / open rules at edge
// nodes, and LDS reads of a ghost neighbour take the nearest lattice node's
// values with the ghost temperature / velocity rule.
#include "lbpc_device.h"

namespace lbpc {

template <int P, bool GEN>
__global__ __launch_bounds__(BLOCK, 2) void k_step(StepParams p) {
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
  const int X0 = blockIdx.x * p.W, X1 = min(X0 + p.W, nx);
  const int Y0 = blockIdx.y * p.H, Y1 = min(Y0 + p.H, ny);
  const int c = X0 - HALO + t;  // unwrapped column of this thread

  const S* __restrict__ fin = static_cast<const S*>(p.fin);
  const S* __restrict__ gin = static_cast<const S*>(p.gin);
  S* __restrict__ fout = static_cast<S*>(p.fout);
  S* __restrict__ gout = static_cast<S*>(p.gout);
  C* __restrict__ phiv = static_cast<C*>(p.phi);

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

  // shifts of the shifted storage forms
  C fsh[Q], gsh[Q];
  storage_shifts<P>(p, fsh, gsh);

  // rates in compute precision
  C sf[Q], sg[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    sf[a] = C(p.s_f[a]);
    sg[a] = C(p.s_g[a]);
  }

  // register queues: pulled f of row r-1, pulled g of rows r-1 and r-2
  C fq1[Q], gq1[Q], gq2[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) fq1[a] = gq1[a] = gq2[a] = C(0);
  C jx1 = C(0), jy1 = C(0);

  const int rbeg = Y0 - 2, rend = Y1 + 2;
  for (int r = rbeg; r < rend; ++r) {
    const int i = r - rbeg;
    const int sl0 = i % RING;                // slot of row r
    const int sl1 = (i + RING - 1) % RING;   // row r-1
    const int sl2 = (i + RING - 2) % RING;   // row r-2
    const int sl3 = (i + RING - 3) % RING;   // row r-3

    // ------------------------------------------------------------ A(r)
    C fn[Q], gn[Q];
    C jxn = C(0), jyn = C(0);
    {
      int rw = r;
      bool ghostr = false;
      if (r < 0 || r >= ny) {
        if (p.pery)
          rw = r < 0 ? r + ny : r - ny;
        else
          ghostr = true;
      }
#pragma unroll
      for (int a = 0; a < Q; ++a) fn[a] = gn[a] = C(0);
      if (doA && !ghostr) {
        pull_node<P, GEN>(p, fin, gin, cw, rw, fsh, gsh, fn, gn);
        C sa = fn[1] + fn[2] + fn[3] + fn[4];
        C sd = fn[5] + fn[6] + fn[7] + fn[8];
        C rho = fn[0] + sa + sd;
        jxn = (fn[1] - fn[3]) + (fn[5] - fn[6] - fn[7] + fn[8]);
        jyn = (fn[2] - fn[4]) + (fn[5] + fn[6] - fn[7] - fn[8]);
        C T = gn[0] + (gn[1] + gn[2] + gn[3] + gn[4]) +
              (gn[5] + gn[6] + gn[7] + gn[8]);
        double psi = pseudo_psi(p, (double)rho, (double)T);
        s_rho[sl0][t] = rho;
        s_T[sl0][t] = T;
        s_psi[sl0][t] = C(psi);
      }
    }
    __syncthreads();

    // ------------------------------------------------ B(r-1) and C1(r-1)
    {
      const int rb = r - 1;
      bool ghostr = (rb < 0 || rb >= ny) && !p.pery;
      if (doB && !ghostr && r >= Y0) {
        // psi rows rb-1, rb, rb+1 (clamped at non-periodic y sides)
        int sm = sl2, sp = sl0;
        if (GEN && !p.pery) {
          if (rb - 1 < 0) sm = sl1;
          if (rb + 1 >= ny) sp = sl1;
        }
        const C pc = s_psi[sl1][t];
        const C pE = s_psi[sl1][ttp], pW = s_psi[sl1][ttm];
        const C pN = s_psi[sp][t], pS = s_psi[sm][t];
        const C pNE = s_psi[sp][ttp], pNW = s_psi[sp][ttm];
        const C pSE = s_psi[sm][ttp], pSW = s_psi[sm][ttm];
        const C sx = C(1.0 / 3.0) * (pE - pW) +
                     C(1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
        const C sy = C(1.0 / 3.0) * (pN - pS) +
                     C(1.0 / 12.0) * ((pNE - pSE) + (pNW - pSW));
        const C mG = C(-p.G);
        const C Fmx = mG * pc * sx, Fmy = mG * pc * sy;
        const C rho = s_rho[sl1][t];
        const C drho = rho - C(p.rho_ave);
        const C Fx = Fmx + drho * C(p.gx), Fy = Fmy + drho * C(p.gy);
        const C vx = (jx1 + C(0.5) * Fx) / rho;
        const C vy = (jy1 + C(0.5) * Fy) / rho;
        s_vx[sl1][t] = vx;
        s_vy[sl1][t] = vy;

        if (doC && rb >= Y0 && rb < Y1) {
          // flow MRT collision with the forcing scheme of the flow model
          C m[Q], ms[Q], fo[Q];
          to_moments(fq1, m);
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
          const C Fm2 = Fmx * Fmx + Fmy * Fmy;
          const C psi2 = pc * pc;
          const C sig12 = C(12.0 * p.sigma);
          C Sf[Q];
          Sf[0] = C(0);
          Sf[1] = C(6) * vF + sig12 * Fm2 / (psi2 * (C(1) / sf[1] - C(0.5)));
          Sf[2] = -C(6) * vF - sig12 * Fm2 / (psi2 * (C(1) / sf[2] - C(0.5)));
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
          const long long o = (long long)rb * nx + c;
#pragma unroll
          for (int a = 0; a < Q; ++a) Tr::st(fout, a * N + o, fo[a] - fsh[a]);
        }
      }
    }
    __syncthreads();

    // -------------------------------------------------------------- C2(r-2)
    {
      const int yc = r - 2;
      if (doC && yc >= Y0 && yc < Y1) {
        const C T = s_T[sl2][t];
        const C rho = s_rho[sl2][t];
        const C vx = s_vx[sl2][t], vy = s_vy[sl2][t];
        // neighbour values (E, W, N, S, NE, NW, SE, SW)
        C Tn[8], vxn[8], vyn[8], rn[8];
        const bool edge = GEN && ((!p.perx && (c == 0 || c == nx - 1)) ||
                                  (!p.pery && (yc == 0 || yc == ny - 1)));
        constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
        constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
        if (!edge) {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const int tt = DX[k] > 0 ? ttp : (DX[k] < 0 ? ttm : t);
            const int sl = DY[k] > 0 ? sl1 : (DY[k] < 0 ? sl3 : sl2);
            Tn[k] = s_T[sl][tt];
            vxn[k] = s_vx[sl][tt];
            vyn[k] = s_vy[sl][tt];
            rn[k] = s_rho[sl][tt];
          }
        } else {
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            Ghost gh = resolve(p, c + DX[k], yc + DY[k]);
            // LDS position: unclamped axes keep their offset, clamped ones
            // fall back to this node's own column / row
            int tt = t + DX[k];
            if (!p.perx && (c + DX[k] < 0 || c + DX[k] >= nx)) tt = t;
            int sl = DY[k] > 0 ? sl1 : (DY[k] < 0 ? sl3 : sl2);
            if (!p.pery && (yc + DY[k] < 0 || yc + DY[k] >= ny)) sl = sl2;
            rn[k] = s_rho[sl][tt];
            if (gh.kind == GH_INSIDE) {
              Tn[k] = s_T[sl][tt];
              vxn[k] = s_vx[sl][tt];
              vyn[k] = s_vy[sl][tt];
            } else {
              Tn[k] = C(gh.T);
              const bool wall = gh.kind == GH_WALL;
              vxn[k] = wall ? C(0) : s_vx[sl][tt];
              vyn[k] = wall ? C(0) : s_vy[sl][tt];
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
        const C rcv = rho * C(p.cv);
        C div_lam_gradT;
        if (p.lambda_mode == 0) {
          div_lam_gradT = C(p.lambda0) * lapT;
        } else {
          const C drx = third * (rn[0] - rn[1]) +
                        twelfth * ((rn[4] - rn[5]) + (rn[6] - rn[7]));
          const C dry = third * (rn[2] - rn[3]) +
                        twelfth * ((rn[4] - rn[6]) + (rn[5] - rn[7]));
          const C cvchi = C(p.cv * p.chi);
          div_lam_gradT = rho * cvchi * lapT + cvchi * (drx * dTx + dry * dTy);
        }
        const C dpdT = C(pr_dpdT(p, (double)rho, (double)T));
        const C phi = div_lam_gradT / rcv - C(p.k_th) * lapT +
                      T * (C(1) - dpdT / rcv) * divv;
        const long long o = (long long)yc * nx + c;
        C S0 = phi;
        if (p.improved) {
          const C prev = p.phi_valid ? phiv[o] : phi;
          S0 = phi + C(0.5) * (phi - prev);
        }
        phiv[o] = phi;
        // improved thermal MRT collision: Eqs. (45), (46), (53)-(55)
        C n[Q], ns[Q], go[Q];
        to_moments(gq2, n);
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
#pragma unroll
        for (int a = 0; a < Q; ++a) Tr::st(gout, a * N + o, go[a] - gsh[a]);
      }
    }

    // rotate the register queues
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      fq1[a] = fn[a];
      gq2[a] = gq1[a];
      gq1[a] = gn[a];
    }
    jx1 = jxn;
    jy1 = jyn;
  }
}

// host-side launcher: one instantiation per storage precision and boundary
// mode (GEN = some side is not periodic)
hipError_t launch_step(const StepParams& p, int prec, hipStream_t s) {
  dim3 grid(p.nbx, (p.ny + p.H - 1) / p.H);
  const bool gen = !(p.perx && p.pery);
#define LBPC_LAUNCH(PR)                                                   \
  if (gen)                                                                \
    hipLaunchKernelGGL((k_step<PR, true>), grid, dim3(BLOCK), 0, s, p);   \
  else                                                                    \
    hipLaunchKernelGGL((k_step<PR, false>), grid, dim3(BLOCK), 0, s, p);
  switch (prec) {
    case 0: LBPC_LAUNCH(0); break;
    case 1: LBPC_LAUNCH(1); break;
    case 2: LBPC_LAUNCH(2); break;
    case 3: LBPC_LAUNCH(3); break;
    default: return hipErrorInvalidValue;
  }
#undef LBPC_LAUNCH
  return hipGetLastError();
}

}  // namespace lbpc
