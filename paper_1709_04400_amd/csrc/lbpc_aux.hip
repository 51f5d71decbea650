// lbpc_aux.hip -- the kernels around the fused step: initial equilibria,
// macroscopic fields at the current time level (rho, v, T), the final pass
// of the FP64 diagnostic reduction and the canonical-state transfers of
// checkpoint / restart.
#include "lbpc_device.h"

namespace lbpc {

constexpr int AUX_BLOCK = 256;

// f = M^-1 m^eq(rho, u) of the flow model, g = M^-1 m^eq(T, u) of Eq. (53)
// (or g = g^eq(T, u) of Eq. (14) for the Gong-Cheng model, of Eq. (29) for
// the BGK form of the improved model), for the nodes [i0, i0 + cnt); the
// host FP64 fields of those nodes sit in `in` as [rho | ux | uy | T], each
// of cnt values.
template <int P>
__global__ __launch_bounds__(AUX_BLOCK) void k_init(StepParams p,
                                                    const double* in,
                                                    long long i0,
                                                    long long cnt) {
  using Tr = Prec<P>;
  using S = typename Tr::S;
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li >= cnt) return;
  const long long i = i0 + li;
  const double rho = in[li], vx = in[cnt + li], vy = in[2 * cnt + li],
               T = in[3 * cnt + li];
  const long long y = i / p.nx;
  const int x = (int)(i - y * p.nx);
  const double v2 = vx * vx + vy * vy;
  double m[Q], f[Q];
  m[0] = rho;
  m[1] = rho * (-2.0 + 3.0 * v2);
  m[2] = rho * (1.0 - 3.0 * v2);
  m[3] = rho * vx;
  m[4] = -rho * vx;
  m[5] = rho * vy;
  m[6] = -rho * vy;
  m[7] = rho * (vx * vx - vy * vy);
  m[8] = rho * vx * vy;
  from_moments(m, f);
  using C = typename Tr::C;
  S* fo = static_cast<S*>(const_cast<void*>(p.fin));
  S* go = static_cast<S*>(const_cast<void*>(p.gin));
  C d[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a)
    d[a] = C(f[a] - (Tr::shift ? w_lat(a) * p.rho_ref : 0.0));
  // paired forms: f waits as its stored images for the (f, g) pairs; the
  // node-referenced FP16 form stores every value against the node's own
  // reference (in the layout an initialisation leaves, each node pulls its
  // own values)
  unsigned int hf[Q];
  float rr[Q], tr[Q];
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    rr[a] = ref_round(float(rho));
    tr[a] = ref_round(float(T));
  }
  if constexpr (P == 4) {
    pack_f_local(d, rr, hf);
  } else if constexpr (Tr::paired) {
    pack_f<P>(d, hf);
  } else {
    store_node<P>(fo, p.nx, y, x, d);
  }
  if (p.gc) {
#pragma unroll
    for (int a = 0; a < Q; ++a) {
      const double eu = EXs[a] * vx + EYs[a] * vy;
      f[a] = w_lat(a) * T * (1.0 + 3.0 * eu + 4.5 * eu * eu - 1.5 * v2);
    }
  } else if (p.bgk) {
    // Eq. (29)
#pragma unroll
    for (int a = 0; a < Q; ++a)
      f[a] = w_lat(a) * T * (1.0 + 3.0 * (EXs[a] * vx + EYs[a] * vy));
  } else {
    m[0] = T;
    m[1] = -2.0 * T;
    m[2] = 2.0 * T;
    m[3] = T * vx;
    m[4] = -T * vx;
    m[5] = T * vy;
    m[6] = -T * vy;
    m[7] = 0.0;
    m[8] = 0.0;
    from_moments(m, f);
  }
#pragma unroll
  for (int a = 0; a < Q; ++a)
    d[a] = C(f[a] - (Tr::shift ? w_rest(p, a) * p.T_ref : 0.0));
  if constexpr (P == 4)
    store_pairs_local(p, fo, const_cast<void*>(p.rin), p.nx, y, x, hf, d, tr,
                      ref_word(float(rho), float(T)));
  else if constexpr (Tr::paired)
    store_pairs<P>(fo, const_cast<void*>(p.rin), p.nx, y, x, hf, d);
  else
    store_node<P>(go, p.nx, y, x, d);
}

// Fields at the current time level, computed band by band of rows (the
// readback needs only a band's worth of scratch): the band holds rows
// y0 - 1 ... y0 + nr (one halo row each side, wrapped on a periodic y axis,
// clamped otherwise), and local row j of the band is lattice row
// y0 - 1 + j after that wrap or clamp; m = (nr + 2) nx values per field.

// moments: out = [rho | jx | jy | T | psi], FP64, for the band's rows
template <int P, bool GEN>
__global__ __launch_bounds__(AUX_BLOCK) void k_macro1(StepParams p,
                                                      double* out, int y0,
                                                      int nr) {
  using Tr = Prec<P>;
  using C = typename Tr::C;
  const long long bm = (long long)(nr + 2) * p.nx;
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li >= bm) return;
  const int x = (int)(li % p.nx);
  const int y = wrap_or_clamp(y0 - 1 + (int)(li / p.nx), p.ny, p.pery != 0);
  C fn[Q], gn[Q];
  const Shift<P> sh(p);
  pull_node<P, GEN>(p, static_cast<const typename Tr::S*>(p.fin),
                    static_cast<const typename Tr::S*>(p.gin), x, y, sh,
                    fn, gn);
  C m[Q];
  to_moments(fn, m);
  const C T = gn[0] + (gn[1] + gn[2] + gn[3] + gn[4]) +
              (gn[5] + gn[6] + gn[7] + gn[8]);
  out[li] = (double)m[0];
  out[bm + li] = (double)m[3];
  out[2 * bm + li] = (double)m[5];
  out[3 * bm + li] = (double)T;
  out[4 * bm + li] = pseudo_psi(p, (double)m[0], (double)T);
}

// force and velocity v = (j + F/2)/rho of the band's own rows y0 ...
// y0 + nr - 1 (local rows 1 ... nr); overwrites jx, jy with vx, vy.  A
// neighbour's row is found in the band by its distance from the band's
// first row (modulo ny on a periodic y axis, where a band of ny or more rows
// repeats rows): the band holds a copy of every row it may need.
__global__ __launch_bounds__(AUX_BLOCK) void k_macro2(StepParams p,
                                                      double* io, int y0,
                                                      int nr) {
  const long long bm = (long long)(nr + 2) * p.nx;
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li >= (long long)nr * p.nx) return;
  const int x = (int)(li % p.nx);
  const int y = y0 + (int)(li / p.nx);
  const long long i = li + p.nx;  // local index (row 0 is the halo)
  const double* psi = io + 4 * bm;
  double sx = 0.0, sy = 0.0;
  const int DX[8] = {1, 0, -1, 0, 1, -1, -1, 1};
  const int DY[8] = {0, 1, 0, -1, 1, 1, -1, -1};
  for (int k = 0; k < 8; ++k) {
    Ghost gh = resolve(p, x + DX[k], y + DY[k]);
    const double w = k < 4 ? 1.0 / 3.0 : 1.0 / 12.0;
    const int j = p.pery ? ((gh.y - (y0 - 1)) % p.ny + p.ny) % p.ny
                         : gh.y - (y0 - 1);
    const long long n = (long long)j * p.nx + gh.x;
    const double pn = p.wet && gh.kind == GH_WALL
                          ? wall_psi(p, io[n], io[3 * bm + n])
                          : psi[n];
    sx += w * pn * DX[k];
    sy += w * pn * DY[k];
  }
  const double rho = io[i];
  double Fx = -p.G * psi[i] * sx + (rho - p.rho_ave) * p.gx;
  double Fy = -p.G * psi[i] * sy + (rho - p.rho_ave) * p.gy;
  io[bm + i] = (io[bm + i] + 0.5 * Fx) / rho;
  io[2 * bm + i] = (io[2 * bm + i] + 0.5 * Fy) / rho;
}

// Final pass of the diagnostics: block c reduces the tile records
// [lo_c, hi_c) of lattice c (8 FP64 values each: six sums, then two maxima)
// into out[c]; ranges holds (lo_c, hi_c) pairs, or is NULL for one lattice
// with records [lo, hi).  Each thread takes a fixed strided subset in order
// and the block combines them by a fixed tree, so the result does not depend
// on scheduling.
__global__ __launch_bounds__(AUX_BLOCK) void k_diag_reduce(
    const double* __restrict__ part, const int* __restrict__ ranges, int lo0,
    int hi0, double* __restrict__ out) {
  __shared__ double red[8][AUX_BLOCK];
  const int c = blockIdx.x, t = threadIdx.x;
  const int lo = ranges ? ranges[2 * c] : lo0;
  const int hi = ranges ? ranges[2 * c + 1] : hi0;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int i = lo + t; i < hi; i += AUX_BLOCK) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const double v = part[(long long)i * 8 + k];
      acc[k] = k >= 6 ? (v > acc[k] ? v : acc[k]) : acc[k] + v;
    }
  }
#pragma unroll
  for (int k = 0; k < 8; ++k) red[k][t] = acc[k];
  __syncthreads();
  for (int st = AUX_BLOCK / 2; st > 0; st >>= 1) {
    if (t < st) {
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        const double o = red[k][t + st];
        red[k][t] = k >= 6 ? (o > red[k][t] ? o : red[k][t]) : red[k][t] + o;
      }
    }
    __syncthreads();
  }
  if (t < 8) out[(long long)c * 8 + t] = red[t][0];
}

// canonical FP64 f(t) (which = 0..8) or g(t) (which = 9..17), one direction,
// for the nodes [i0, i0 + cnt) into out[0 .. cnt)
template <int P, bool GEN>
__global__ __launch_bounds__(AUX_BLOCK) void k_canon(StepParams p, int which,
                                                     double* out, long long i0,
                                                     long long cnt) {
  using Tr = Prec<P>;
  using C = typename Tr::C;
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li >= cnt) return;
  const long long i = i0 + li;
  const int x = (int)(i % p.nx), y = (int)(i / p.nx);
  C fn[Q], gn[Q];
  const Shift<P> sh(p);
  pull_node<P, GEN>(p, static_cast<const typename Tr::S*>(p.fin),
                    static_cast<const typename Tr::S*>(p.gin), x, y, sh,
                    fn, gn);
  C v = C(0);
#pragma unroll
  for (int a = 0; a < Q; ++a) {
    if (which == a) v = fn[a];
    if (which == Q + a) v = gn[a];
  }
  out[li] = (double)v;
}

// FP64 canonical direction `which` of the nodes [i0, i0 + cnt), held in
// in[0 .. cnt) -> storage buffer (fresh layout).  The node-referenced FP16
// form needs each node's reference before its directions 1-8: the rest
// populations, which the host loads first (which = 0 before 1-8, 9 before
// 10-17), give it, rho_ref = f_0 / w_0 and T_ref = g_0 / wg_0 in binary16.
template <int P>
__global__ __launch_bounds__(AUX_BLOCK) void k_load(StepParams p, int which,
                                                    const double* in,
                                                    long long i0,
                                                    long long cnt) {
  using Tr = Prec<P>;
  using S = typename Tr::S;
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li >= cnt) return;
  const long long i = i0 + li;  // node; its value is in[li]
  const int a = which % Q;
  const long long y = i / p.nx;
  const long long o = dix(p.nx, a, y, (int)(i - y * p.nx));
  if constexpr (P == 3) {
    // FP16 deviation form: f is the low half (the first of the pair in
    // memory), g the high half, of the (f, g) word of direction a, and the
    // rest populations an FP32 (f_0, g_0) pair per node
    const int half = which < Q ? 0 : 1;
    const double sh = which < Q ? w_lat(a) * p.rho_ref : w_rest(p, a) * p.T_ref;
    if (a == 0) {
      float* rest = static_cast<float*>(const_cast<void*>(p.rin));
      rest[2 * i + half] = float(in[li] - sh);
    } else {
      unsigned short* h =
          static_cast<unsigned short*>(const_cast<void*>(p.fin));
      h[2 * o + half] = __half_as_ushort(__float2half_rn(float(in[li] - sh)));
    }
    return;
  } else if constexpr (P == 4) {
    const int half = which < Q ? 0 : 1;
    unsigned short* h = static_cast<unsigned short*>(const_cast<void*>(p.fin));
    const long long o0 = dix(p.nx, 0, y, (int)(i - y * p.nx));
    if (a == 0) {
      float* rest = static_cast<float*>(const_cast<void*>(p.rin));
      rest[2 * i + half] = float(in[li]);
      const double w0 = which < Q ? w_lat(0) : w_rest(p, 0);
      h[2 * o0 + half] = __half_as_ushort(__float2half_rn(float(in[li] / w0)));
    } else {
      const float ref = __half2float(__ushort_as_half(h[2 * o0 + half]));
      const float wr = which < Q ? float(w_lat(a)) * ref
                                 : float(w_rest(p, a)) * ref;
      h[2 * o + half] = __half_as_ushort(__float2half_rn(float(in[li]) - wr));
    }
    return;
  } else if constexpr (Tr::paired) {
    // FP32 forms: f first, g second, in the (f, g) pair of direction a
    const double sh = !Tr::shift ? 0.0
                      : which < Q ? w_lat(a) * p.rho_ref
                                  : w_rest(p, a) * p.T_ref;
    float* w = static_cast<float*>(const_cast<void*>(p.fin));
    w[2 * o + (which < Q ? 0 : 1)] = float(in[li] - sh);
  } else if (which < Q) {
    S* fo = static_cast<S*>(const_cast<void*>(p.fin));
    fo[o] = in[li];
  } else {
    S* go = static_cast<S*>(const_cast<void*>(p.gin));
    go[o] = in[li];
  }
}

// phi history between its compute precision and FP64
// (nodes [i0, i0 + cnt); `out` / `in` hold that chunk)
template <class C>
__global__ __launch_bounds__(AUX_BLOCK) void k_phi_out(long long i0,
                                                       long long cnt,
                                                       const C* phi,
                                                       double* out) {
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li < cnt) out[li] = (double)phi[i0 + li];
}
template <class C>
__global__ __launch_bounds__(AUX_BLOCK) void k_phi_in(long long i0,
                                                      long long cnt, C* phi,
                                                      const double* in) {
  const long long li = (long long)blockIdx.x * AUX_BLOCK + threadIdx.x;
  if (li < cnt) phi[i0 + li] = C(in[li]);
}

// ------------------------------------------------------------- launchers

static inline unsigned nblocks(long long N) {
  return (unsigned)((N + AUX_BLOCK - 1) / AUX_BLOCK);
}

#define LBPC_PREC_SWITCH(prec, X) \
  switch (prec) {                 \
    case 0: X(0); break;          \
    case 1: X(1); break;          \
    case 2: X(2); break;          \
    case 3: X(3); break;          \
    case 4: X(4); break;          \
    default: return hipErrorInvalidValue; \
  }

hipError_t launch_init(const StepParams& p, int prec, const double* in,
                       long long i0, long long cnt, hipStream_t s) {
#define X(PR) hipLaunchKernelGGL(k_init<PR>, dim3(nblocks(cnt)), dim3(AUX_BLOCK), 0, s, p, in, i0, cnt)
  LBPC_PREC_SWITCH(prec, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_macro(const StepParams& p, int prec, double* io, int y0,
                        int nr, hipStream_t s) {
  const bool gen = !(p.perx && p.pery);
  const long long m = (long long)(nr + 2) * p.nx;
#define X(PR)                                                                    \
  if (gen)                                                                       \
    hipLaunchKernelGGL((k_macro1<PR, true>), dim3(nblocks(m)), dim3(AUX_BLOCK), 0, s, p, io, y0, nr); \
  else                                                                           \
    hipLaunchKernelGGL((k_macro1<PR, false>), dim3(nblocks(m)), dim3(AUX_BLOCK), 0, s, p, io, y0, nr);
  LBPC_PREC_SWITCH(prec, X)
#undef X
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_macro2, dim3(nblocks((long long)nr * p.nx)),
                     dim3(AUX_BLOCK), 0, s, p, io, y0, nr);
  return hipGetLastError();
}

hipError_t launch_diag_reduce(const double* part, const int* ranges, int lo,
                              int hi, int nlat, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag_reduce, dim3(nlat), dim3(AUX_BLOCK), 0, s, part,
                     ranges, lo, hi, out);
  return hipGetLastError();
}

hipError_t launch_canon(const StepParams& p, int prec, int which, double* out,
                        long long i0, long long cnt, hipStream_t s) {
  const bool gen = !(p.perx && p.pery);
#define X(PR)                                                                    \
  if (gen)                                                                       \
    hipLaunchKernelGGL((k_canon<PR, true>), dim3(nblocks(cnt)), dim3(AUX_BLOCK), 0, s, p, which, out, i0, cnt); \
  else                                                                           \
    hipLaunchKernelGGL((k_canon<PR, false>), dim3(nblocks(cnt)), dim3(AUX_BLOCK), 0, s, p, which, out, i0, cnt);
  LBPC_PREC_SWITCH(prec, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_load(const StepParams& p, int prec, int which,
                       const double* in, long long i0, long long cnt,
                       hipStream_t s) {
#define X(PR) hipLaunchKernelGGL(k_load<PR>, dim3(nblocks(cnt)), dim3(AUX_BLOCK), 0, s, p, which, in, i0, cnt)
  LBPC_PREC_SWITCH(prec, X)
#undef X
  return hipGetLastError();
}

hipError_t launch_phi_out(const StepParams& p, int prec, double* out,
                          long long i0, long long cnt, hipStream_t s) {
  if (prec == 0)
    hipLaunchKernelGGL(k_phi_out<double>, dim3(nblocks(cnt)), dim3(AUX_BLOCK),
                       0, s, i0, cnt, static_cast<const double*>(p.phi), out);
  else
    hipLaunchKernelGGL(k_phi_out<float>, dim3(nblocks(cnt)), dim3(AUX_BLOCK),
                       0, s, i0, cnt, static_cast<const float*>(p.phi), out);
  return hipGetLastError();
}

hipError_t launch_phi_in(const StepParams& p, int prec, const double* in,
                         long long i0, long long cnt, hipStream_t s) {
  if (prec == 0)
    hipLaunchKernelGGL(k_phi_in<double>, dim3(nblocks(cnt)), dim3(AUX_BLOCK),
                       0, s, i0, cnt, static_cast<double*>(p.phi), in);
  else
    hipLaunchKernelGGL(k_phi_in<float>, dim3(nblocks(cnt)), dim3(AUX_BLOCK),
                       0, s, i0, cnt, static_cast<float*>(p.phi), in);
  return hipGetLastError();
}

}  // namespace lbpc
