// lbpc_step2.hip -- two coupled time steps per launch for the 4-byte storage
// forms on periodic lattices.
//
// The single-step kernel moves every node's whole state through HBM once
// per step, so it cannot beat the memory time of that traffic.  This kernel
// runs two steps in one row march: step 1 pulls f*(t-1), g*(t-1) from HBM
// and, instead of storing f*(t), g*(t), keeps them in LDS rings; step 2
// trails it by a few rows, pulls from those rings and stores f*(t+1),
// g*(t+1) to HBM.  The bytes per node and launch are those of one step, for
// two steps.  Each step evaluates the single-step kernel's expressions (the
// compiler fuses some multiply-adds differently here, so the results agree
// with two single-step launches to FP32 rounding, not bitwise).
//
// Geometry (one block of TS_BLOCK threads, one column each, on a strip of W
// columns and a run of H rows; "dir" is the march direction):
//   step 1, A / B / C on the strip plus 5 / 4 / 3 columns and rows beyond it
//     (step 2 pulls f*(t), g*(t) one node beyond its own A range, which is
//     2 beyond the strip; step 1's C needs B one further, B needs A);
//   step 2, A / B / C on the strip plus 2 / 1 / 0.
// One iteration handles three stages separated by barriers:
//   X: step-1 A of row r;        step-2 B of row r - 6 dir (stores f*(t+1))
//   Y: step-1 B of row r - dir;  step-2 C of row r - 7 dir (stores g*(t+1),
//      phi(t+1)); the history phi(t-1) of row r - 2 dir and the pull of row
//      r + dir are issued here
//   Z: step-1 C of row r - 2 dir; step-2 A of row r - 4 dir
// so every stage reads only what an earlier stage wrote.  Step 1's f*(t)
// rows stay in LDS for 5 iterations and g*(t) rows for 4; step 2 keeps its
// pulled values in registers until its collisions use them, and phi(t) of
// its row (computed by step 1 five iterations earlier) likewise.
#include "lbpc_device.h"

namespace lbpc {

constexpr int TS_BLOCK = 256;
constexpr int TS_HALO = 5;
constexpr int TS_FR = 5;   // rows of f*(t) kept in LDS
constexpr int TS_GR = 4;   // rows of g*(t) kept in LDS

// Peng-Robinson EOS of Eq. (56) in the FP32 arithmetic (the cancelling
// combinations in FP64): psi and T (dp/dT)_rho; the same expressions as the
// single-step kernel.
__device__ __forceinline__ void ts_eos(const StepParams& p, float rho, float T,
                                       float& psi_out, float& tdp,
                                       bool& valid) {
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
  const double psi = fsqrt(float(psi2 > 0.0 ? psi2 : 0.0));
  tdp = float((rRT + ar2 * (p.kappa * (double)(s * sq))) * (double)inv);
  valid = psi2 >= 0.0 && rd > 0.0 && rd * p.b < 1.0 && T - T == 0.0f;
  psi_out = float(psi);
}

// Interaction force, buoyancy and velocity from the psi ring (rows sm, sl,
// sp = the row below, the row, the row above in lattice terms).
struct TsForce {
  float sx, sy, Fx, Fy, vx, vy, irn, rho;
};
__device__ __forceinline__ TsForce ts_force(const StepParams& p,
                                            const float (*s_psi)[TS_BLOCK],
                                            const float (*s_rho)[TS_BLOCK],
                                            int sm, int sl, int sp, int t,
                                            float jx, float jy) {
  using C = float;
  const int ttm = t - 1, ttp = t + 1;
  const C pc = s_psi[sl][t];
  const C pE = s_psi[sl][ttp], pW = s_psi[sl][ttm];
  const C pN = s_psi[sp][t], pS = s_psi[sm][t];
  const C pNE = s_psi[sp][ttp], pNW = s_psi[sp][ttm];
  const C pSE = s_psi[sm][ttp], pSW = s_psi[sm][ttm];
  TsForce f;
  f.sx = C(1.0 / 3.0) * (pE - pW) +
         C(1.0 / 12.0) * ((pNE - pNW) + (pSE - pSW));
  f.sy = C(1.0 / 3.0) * (pN - pS) +
         C(1.0 / 12.0) * ((pNE - pSE) + (pNW - pSW));
  const C mGpc = C(-p.G) * pc;
  const C Fmx = mGpc * f.sx, Fmy = mGpc * f.sy;
  const C rho = s_rho[sl][t];
  const C drho = rho - C(p.rho_ave);
  f.Fx = Fmx + drho * C(p.gx);
  f.Fy = Fmy + drho * C(p.gy);
  f.irn = recip(rho);
  f.vx = (jx + C(0.5) * f.Fx) * f.irn;
  f.vy = (jy + C(0.5) * f.Fy) * f.irn;
  f.rho = rho;
  return f;
}

// Flow MRT collision with the forcing scheme; fb pulled values, fo output.
__device__ __forceinline__ void ts_flow(const StepParams& p, const float sf[Q],
                                        const float fb[Q], const TsForce& F,
                                        float fo[Q]) {
  using C = float;
  C m[Q], ms[Q];
  to_moments(fb, m);
  const C rho = F.rho, vx = F.vx, vy = F.vy, Fx = F.Fx, Fy = F.Fy;
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
  const C s2 = F.sx * F.sx + F.sy * F.sy;
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
    ms[k] = m[k] - sf[k] * (m[k] - meq[k]) + (C(1) - C(0.5) * sf[k]) * Sf[k];
  from_moments(ms, fo);
}

// Thermal source phi of Eq. (28) from the T, v (and rho) rings: rows sS,
// sl, sN below / at / above the node.
__device__ __forceinline__ float ts_phi(const StepParams& p,
                                        const float (*s_T)[TS_BLOCK],
                                        const float (*s_vx)[TS_BLOCK],
                                        const float (*s_vy)[TS_BLOCK],
                                        const float (*s_rho)[TS_BLOCK],
                                        int sS, int sl, int sN, int t,
                                        float tdp, float irq, float& T_out,
                                        float& vx_out, float& vy_out) {
  using C = float;
  const C T = s_T[sl][t];
  const C vx = s_vx[sl][t], vy = s_vy[sl][t];
  C Tn[8], vxn[8], vyn[8], rn[8];
  constexpr int DX[8] = {1, -1, 0, 0, 1, -1, 1, -1};
  constexpr int DY[8] = {0, 0, 1, -1, 1, 1, -1, -1};
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const int tt = t + DX[k];
    const int s = DY[k] > 0 ? sN : (DY[k] < 0 ? sS : sl);
    Tn[k] = s_T[s][tt];
    vxn[k] = s_vx[s][tt];
    vyn[k] = s_vy[s][tt];
    rn[k] = p.lambda_mode ? s_rho[s][tt] : C(0);
  }
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
  C lam_term;
  if (p.lambda_mode == 0) {
    lam_term = C(p.lam_over_cv) * irq * lapT;
  } else {
    const C drx = third * (rn[0] - rn[1]) +
                  twelfth * ((rn[4] - rn[5]) + (rn[6] - rn[7]));
    const C dry = third * (rn[2] - rn[3]) +
                  twelfth * ((rn[4] - rn[6]) + (rn[5] - rn[7]));
    lam_term = C(p.chi) * (lapT + irq * (drx * dTx + dry * dTy));
  }
  T_out = T;
  vx_out = vx;
  vy_out = vy;
  return lam_term - C(p.k_th) * lapT + (T - tdp * irq * C(p.inv_cv)) * divv;
}

// Improved (or compromised) thermal MRT collision, Eqs. (45), (46),
// (53)-(55).
__device__ __forceinline__ void ts_thermal(const StepParams& p,
                                           const float sg[Q],
                                           const float gb[Q], float T,
                                           float vx, float vy, float S0,
                                           float go[Q]) {
  using C = float;
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

template <int P>
__device__ __forceinline__ void two_step_tile(const StepParams& p, int bx,
                                              int by) {
  static_assert(P == 1 || P == 2, "two steps per launch: 4-byte forms");
  using Tr = Prec<P>;
  using S = typename Tr::S;
  using C = float;
  using R = float;
  constexpr int B = TS_BLOCK;

  // step-1 and step-2 rings of rho, T, psi, vx, vy (RING rows each)
  __shared__ C a_rho[RING][B], a_T[RING][B], a_psi[RING][B], a_vx[RING][B],
      a_vy[RING][B];
  __shared__ C b_rho[RING][B], b_T[RING][B], b_psi[RING][B], b_vx[RING][B],
      b_vy[RING][B];
  // step 1's post-collision f*(t), g*(t) (storage form: deviations for the
  // shifted form, converted back when step 2 pulls them)
  __shared__ C o_f[TS_FR][Q][B];
  __shared__ C o_g[TS_GR][Q][B];

  const int t = threadIdx.x;
  const int nx = p.nx, ny = p.ny;
  const int X0 = bx * p.W, X1 = min(X0 + p.W, nx);
  const int Y0 = by * p.H, Y1 = min(Y0 + p.H, ny);
  const int c = X0 - TS_HALO + t;
  int cw = c < 0 ? c + nx : (c >= nx ? c - nx : c);
  const int cl = cw < 0 ? 0 : (cw >= nx ? nx - 1 : cw);
  // column roles (unwrapped columns relative to the strip)
  const bool doA1 = c < X1 + 5;
  const bool doB1 = c >= X0 - 4 && c < X1 + 4;
  const bool doC1 = c >= X0 - 3 && c < X1 + 3;
  const bool doA2 = c >= X0 - 2 && c < X1 + 2;
  const bool doB2 = c >= X0 - 1 && c < X1 + 1;
  const bool doC2 = c >= X0 && c < X1;

  const S* __restrict__ fin = static_cast<const S*>(p.fin);
  const S* __restrict__ gin = static_cast<const S*>(p.gin);
  S* __restrict__ fout = static_cast<S*>(p.fout);
  const Gbl<C>* __restrict__ phiv = gbl(static_cast<const C*>(p.phi));
  Gbl<C>* __restrict__ phio = gbl(static_cast<C*>(p.phi_out));

  const Shift<P> sh(p);
  C sf[Q], sg[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    sf[a] = C(p.s_f[a]);
    sg[a] = C(p.s_g[a]);
  }

  auto wrap_row = [&](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
  // rows of a stage's range, in absolute lattice terms (unwrapped)
  auto in_rows = [&](int row, int ext) {
    return row >= Y0 - ext && row < Y1 + ext;
  };

  const int dir = (by & 1) ? -1 : 1;
  const int nit = Y1 - Y0 + 12;
  const int rfirst = dir > 0 ? Y0 - 5 : Y1 + 4;
  const int rlast = rfirst + dir * (nit - 1);
  auto pull_row = [&](int rt, R* fr, R* gr) {
    const int rc = dir > 0 ? min(rt, rlast) : max(rt, rlast);
    pull_raw<P, false>(p, fin, gin, cl, wrap_row(rc), fr, gr);
  };

  // step-1 queues of pulled values (one row of prefetch)
  R F[Q], G[Q], fq1[Q], gq1[Q], gq2[Q];
  // step-2 queues: pulled f for B (2 rows), pulled g for C (3 rows), j (2),
  // T dp/dT (3), 1/rho (1), and phi(t) of its node from step 1 (5)
  C f2a[Q], f2b[Q], g2a[Q], g2b[Q], g2c[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    F[a] = G[a] = fq1[a] = gq1[a] = gq2[a] = R(0);
    f2a[a] = f2b[a] = g2a[a] = g2b[a] = g2c[a] = C(0);
  }
  C jx1 = 0, jy1 = 0, tdp1 = 0, tdp2 = 0, irq = 0;              // step 1
  C j2x_a = 0, j2y_a = 0, j2x_b = 0, j2y_b = 0;                  // step 2
  C t2a = 0, t2b = 0, t2c = 0, irq2 = 0;
  C ph1 = 0, ph2 = 0, ph3 = 0, ph4 = 0, ph5 = 0;
  // step-2 f* of a row waits one iteration for g* of that row: the (f, g)
  // pairs are stored together
  unsigned int hf1[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) hf1[a] = 0u;

  pull_row(rfirst, F, G);

  for (int it = 0; it < nit; ++it) {
    const int r = rfirst + dir * it;
    // ring slots: a row's slot is the iteration that wrote it, mod RING
    auto sl = [&](int back) { return (it - back + 2 * RING) % RING; };
    unsigned int hfn[Q];  // step-2 f* of row r - 6 dir
#pragma unroll
    for (int a = 0; a < Q; ++a) hfn[a] = hf1[a];

    // ---------------------------------------------------------- stage X
    C jxn = 0, jyn = 0, tdpn = 0;
    if (doA1 && in_rows(r, 5)) {                  // step-1 A(r)
      C fa[Q], ga[Q];
      cook_f<P, false>(p, sh, cw, wrap_row(r), F, G, fa);
      cook_g<P, false>(p, sh, cw, wrap_row(r), F, G, ga);
      const C sa = fa[1] + fa[2] + fa[3] + fa[4];
      const C sd = fa[5] + fa[6] + fa[7] + fa[8];
      const C rho = fa[0] + sa + sd;
      jxn = (fa[1] - fa[3]) + (fa[5] - fa[6] - fa[7] + fa[8]);
      jyn = (fa[2] - fa[4]) + (fa[5] + fa[6] - fa[7] - fa[8]);
      const C T = ga[0] + (ga[1] + ga[2] + ga[3] + ga[4]) +
                  (ga[5] + ga[6] + ga[7] + ga[8]);
      C psi;
      bool valid;
      ts_eos(p, rho, T, psi, tdpn, valid);
      if (!valid) *p.bad = 1;
      a_rho[sl(0)][t] = rho;
      a_T[sl(0)][t] = T;
      a_psi[sl(0)][t] = psi;
    }
    C irn2 = 0;
    {                                              // step-2 B(r - 6 dir)
      const int rb = r - 6 * dir;
      if (doB2 && in_rows(rb, 1)) {
        // psi2 rows: r-5dir, r-6dir, r-7dir were written by step-2 A at
        // iterations it-1, it-2, it-3
        const int sm = dir > 0 ? sl(3) : sl(1), sp = dir > 0 ? sl(1) : sl(3);
        const TsForce Fo = ts_force(p, b_psi, b_rho, sm, sl(2), sp, t, j2x_b,
                                    j2y_b);
        irn2 = Fo.irn;
        b_vx[sl(2)][t] = Fo.vx;
        b_vy[sl(2)][t] = Fo.vy;
        if (doC2 && in_rows(rb, 0)) {
          C fo[Q];
          ts_flow(p, sf, f2b, Fo, fo);
#pragma unroll
          for (int a = 0; a < Q; ++a) fo[a] -= sh.f(a);
          pack_f<P>(fo, hfn);
        }
      }
    }
    __syncthreads();

    // ---------------------------------------------------------- stage Y
    C irn = 0;
    {                                              // step-1 B(r - dir)
      const int rb = r - dir;
      if (doB1 && in_rows(rb, 4)) {
        const int sm = dir > 0 ? sl(2) : sl(0), sp = dir > 0 ? sl(0) : sl(2);
        const TsForce Fo = ts_force(p, a_psi, a_rho, sm, sl(1), sp, t, jx1,
                                    jy1);
        irn = Fo.irn;
        a_vx[sl(1)][t] = Fo.vx;
        a_vy[sl(1)][t] = Fo.vy;
        if (doC1 && in_rows(rb, 3)) {
          C fb[Q], fo[Q];
          cook_f<P, false>(p, sh, cw, wrap_row(rb), fq1, fq1, fb);
          ts_flow(p, sf, fb, Fo, fo);
          // f*(t) of row r - dir into its LDS row (storage form)
#pragma unroll
          for (int a = 0; a < Q; ++a)
            o_f[(it + 4 * TS_FR - 1) % TS_FR][a][t] = fo[a] - sh.f(a);
        }
      }
    }
    // history phi(t-1) of the row step-1 C takes next, before the prefetch
    C hphi = 0;
    {
      const int yc = r - 2 * dir;
      if (doC1 && in_rows(yc, 3) && p.phi_valid && p.improved)
        hphi = phiv[(long long)wrap_row(yc) * nx + cw];
    }
    R gn[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      fq1[a] = F[a];
      gn[a] = R(0);
    }
    pull_row(r + dir, F, gn);
    {                                              // step-2 C(r - 7 dir)
      const int yc = r - 7 * dir;
      if (doC2 && in_rows(yc, 0)) {
        const int sN = dir > 0 ? sl(2) : sl(4), sS = dir > 0 ? sl(4) : sl(2);
        C T, vx, vy;
        const C phi = ts_phi(p, b_T, b_vx, b_vy, b_rho, sS, sl(3), sN, t, t2c,
                             irq2, T, vx, vy);
        C S0 = phi;
        if (p.improved) S0 = phi + C(0.5) * (phi - ph5);
        phio[(long long)yc * nx + c] = phi;
        C go[Q];
        ts_thermal(p, sg, g2c, T, vx, vy, S0, go);
#pragma unroll
        for (int a = 0; a < Q; ++a) go[a] -= sh.g(a);
        store_pairs<P>(fout, nullptr, nx, yc, c, hf1, go);
      }
    }
    __syncthreads();

    // ---------------------------------------------------------- stage Z
    C phin = 0;
    {                                              // step-1 C(r - 2 dir)
      const int yc = r - 2 * dir;
      if (doC1 && in_rows(yc, 3)) {
        const int sN = dir > 0 ? sl(1) : sl(3), sS = dir > 0 ? sl(3) : sl(1);
        C T, vx, vy;
        const C phi = ts_phi(p, a_T, a_vx, a_vy, a_rho, sS, sl(2), sN, t,
                             tdp2, irq, T, vx, vy);
        C S0 = phi;
        if (p.improved) {
          const C prev = p.phi_valid ? hphi : phi;
          S0 = phi + C(0.5) * (phi - prev);
        }
        phin = phi;
        C gb[Q], go[Q];
        cook_g<P, false>(p, sh, c, yc, gq2, gq2, gb);
        ts_thermal(p, sg, gb, T, vx, vy, S0, go);
#pragma unroll
        for (int a = 0; a < Q; ++a)
          o_g[(it + 4 * TS_GR - 2) % TS_GR][a][t] = go[a] - sh.g(a);
      }
    }
    C j2xn = 0, j2yn = 0, t2n = 0;
    C f2n[Q], g2n[Q];
#pragma unroll
    for (int a = 0; a < Q; ++a) f2n[a] = g2n[a] = C(0);
    {                                              // step-2 A(r - 4 dir)
      const int ya = r - 4 * dir;
      if (doA2 && in_rows(ya, 2)) {
        // pull f*(t), g*(t) from the LDS rows: direction a comes from
        // (x - e_ax, y - e_ay), the row k iterations back in march order
#pragma unroll
        for (int a = 0; a < Q; ++a) {
          const int back = 4 + (dir > 0 ? EYs[a] : -EYs[a]);
          const int tt = t - EXs[a];
          const C fv = o_f[(it - back + 4 * TS_FR) % TS_FR][a][tt];
          const C gv = o_g[(it - back + 4 * TS_GR) % TS_GR][a][tt];
          // as cook_f / cook_g: the shift is added for the shifted form only
          if constexpr (Tr::shift) {
            f2n[a] = fv + sh.f(a);
            g2n[a] = gv + sh.g(a);
          } else {
            f2n[a] = fv;
            g2n[a] = gv;
          }
        }
        const C sa = f2n[1] + f2n[2] + f2n[3] + f2n[4];
        const C sd = f2n[5] + f2n[6] + f2n[7] + f2n[8];
        const C rho = f2n[0] + sa + sd;
        j2xn = (f2n[1] - f2n[3]) + (f2n[5] - f2n[6] - f2n[7] + f2n[8]);
        j2yn = (f2n[2] - f2n[4]) + (f2n[5] + f2n[6] - f2n[7] - f2n[8]);
        const C T = g2n[0] + (g2n[1] + g2n[2] + g2n[3] + g2n[4]) +
                    (g2n[5] + g2n[6] + g2n[7] + g2n[8]);
        C psi;
        bool valid;
        ts_eos(p, rho, T, psi, t2n, valid);
        if (!valid) *p.bad = 1;
        b_rho[sl(0)][t] = rho;
        b_T[sl(0)][t] = T;
        b_psi[sl(0)][t] = psi;
      }
    }
    __syncthreads();

    // rotate the per-column queues
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      gq2[a] = gq1[a];
      gq1[a] = G[a];
      G[a] = gn[a];
      f2b[a] = f2a[a];
      f2a[a] = f2n[a];
      g2c[a] = g2b[a];
      g2b[a] = g2a[a];
      g2a[a] = g2n[a];
    }
    jx1 = jxn;
    jy1 = jyn;
    tdp2 = tdp1;
    tdp1 = tdpn;
    irq = irn;
    j2x_b = j2x_a;
    j2y_b = j2y_a;
    j2x_a = j2xn;
    j2y_a = j2yn;
    t2c = t2b;
    t2b = t2a;
    t2a = t2n;
    irq2 = irn2;
    ph5 = ph4;
    ph4 = ph3;
    ph3 = ph2;
    ph2 = ph1;
    ph1 = phin;
#pragma unroll
    for (int a = 0; a < Q; ++a) hf1[a] = hfn[a];
  }
}

template <int P>
__global__ __launch_bounds__(TS_BLOCK) __attribute__((amdgpu_waves_per_eu(
    1, 1))) void k_two_steps(StepParams p) {
  int bx, by;
  // tiles one XCD runs together are x-neighbours (as in the single step)
  const int nb = p.nbx * p.nby;
  int b = blockIdx.x;
  if (p.xcd_order) {
    const int per = (nb + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    const int full = nb - 8 * (per - 1);
    b = xcd < full ? xcd * per + k : full * per + (xcd - full) * (per - 1) + k;
  }
  by = b / p.nbx;
  bx = b - by * p.nbx;
  two_step_tile<P>(p, bx, by);
}

hipError_t launch_two_steps(const StepParams& p, int prec, hipStream_t s) {
  if (!(p.perx && p.pery) || p.bw != TS_BLOCK || p.W > TS_BLOCK - 2 * TS_HALO)
    return hipErrorInvalidValue;
  const dim3 grid(p.nbx * p.nby);
  if (prec == 1)
    hipLaunchKernelGGL(k_two_steps<1>, grid, dim3(TS_BLOCK), 0, s, p);
  else if (prec == 2)
    hipLaunchKernelGGL(k_two_steps<2>, grid, dim3(TS_BLOCK), 0, s, p);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace lbpc
