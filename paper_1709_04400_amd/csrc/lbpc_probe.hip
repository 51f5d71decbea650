// lbpc_probe.hip -- memory-ceiling probes for the benchmark (not part of the
// step library): what the HBM delivers to (a) streaming copy, read-only and
// write-only kernels and (b) a
// kernel with exactly the fused step's access pattern and no arithmetic, a
// pure pull-stream f_a(x) = f*_a(x - e_a) of both distributions plus the
// phi history, in the same [ny][9][nx] row layout, tile shape, alternating
// row-march direction and one-row-ahead prefetch.  The step moves the same
// algorithmic bytes per launch, so its time over the pattern kernel's is the
// fraction of the reachable bandwidth it attains.
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace {

template <class T> using Gbl = __attribute__((address_space(1))) T;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ long long pix(int nx, int a, long long y, int x) {
  return (y * 9 + a) * nx + x;
}

// Streaming kernels over 16-byte vectors: each thread moves UNR vectors per
// pass (all loads issued before the first store), grid-stride.  NT selects
// non-temporal accesses.
template <int UNR, bool NT>
__global__ __launch_bounds__(256) void k_copy(const u32x4* __restrict__ src,
                                              u32x4* __restrict__ dst,
                                              long long n) {
  const long long step = (long long)gridDim.x * 256 * UNR;
  for (long long base = (long long)blockIdx.x * 256 * UNR + threadIdx.x;
       base < n; base += step) {
    u32x4 v[UNR];
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) v[u] = NT ? __builtin_nontemporal_load(&src[i]) : src[i];
    }
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) {
        if (NT)
          __builtin_nontemporal_store(v[u], &dst[i]);
        else
          dst[i] = v[u];
      }
    }
  }
}

// Read only: the vectors' xor, one 16-byte result per thread (kept so the
// loads are not removed).
template <int UNR>
__global__ __launch_bounds__(256) void k_read(const u32x4* __restrict__ src,
                                              u32x4* __restrict__ out,
                                              long long n) {
  u32x4 acc = {0u, 0u, 0u, 0u};
  const long long step = (long long)gridDim.x * 256 * UNR;
  for (long long base = (long long)blockIdx.x * 256 * UNR + threadIdx.x;
       base < n; base += step) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) {
        const u32x4 v = src[i];
        acc ^= v;
      }
    }
  }
  out[(long long)blockIdx.x * 256 + threadIdx.x] = acc;
}

// Write only.
template <int UNR>
__global__ __launch_bounds__(256) void k_write(u32x4* __restrict__ dst,
                                               long long n) {
  const u32x4 v = {1u, 2u, 3u, 4u};
  const long long step = (long long)gridDim.x * 256 * UNR;
  for (long long base = (long long)blockIdx.x * 256 * UNR + threadIdx.x;
       base < n; base += step) {
#pragma unroll
    for (int u = 0; u < UNR; ++u) {
      const long long i = base + (long long)u * 256;
      if (i < n) dst[i] = v;
    }
  }
}

// Pull-stream with the step's tiling: block of BW threads on a strip of W
// columns (plus 2 halo columns each side) and a run of H rows of a periodic
// nx x ny lattice; the block marches H + 4 rows (2 halo rows each end) in
// the direction alternating with the run index, loads all 18 pulled values
// of every lane, with the next row's loads issued before the current row's
// stores.  Every lane stores every row, so the stores never sit in a branch
// (a branch around them leaves the compiler's wait counts conservative, and
// each row would then wait for the one in flight): lanes and rows outside
// the tile store into a small sink of 19 nx values, which stays in cache.
template <class T, int BW>
__global__ __launch_bounds__(BW) void k_pattern(
    const T* __restrict__ fin, const T* __restrict__ gin,
    T* __restrict__ fout, T* __restrict__ gout, const T* __restrict__ phin,
    T* __restrict__ phout, T* __restrict__ sink, int nx, int ny, int W,
    int H, int nbx) {
  const Gbl<T>* F = (const Gbl<T>*)fin;
  const Gbl<T>* G = (const Gbl<T>*)gin;
  Gbl<T>* FO = (Gbl<T>*)fout;
  Gbl<T>* GO = (Gbl<T>*)gout;
  const Gbl<T>* PI = (const Gbl<T>*)phin;
  Gbl<T>* PO = (Gbl<T>*)phout;
  // tiles one XCD runs together are x-neighbours (as in the step)
  const int nb = gridDim.x;
  int b = blockIdx.x;
  {
    const int per = (nb + 7) / 8;
    const int xcd = b % 8, k = b / 8;
    const int full = nb - 8 * (per - 1);
    b = xcd < full ? xcd * per + k : full * per + (xcd - full) * (per - 1) + k;
  }
  const int by = b / nbx, bx = b - by * nbx;
  const int X0 = bx * W, X1 = min(X0 + W, nx);
  const int Y0 = by * H, Y1 = min(Y0 + H, ny);
  int c = X0 - 2 + (int)threadIdx.x;
  const bool own = c >= X0 && c < X1;
  c = c < 0 ? c + nx : (c >= nx ? c - nx : c);
  if (c < 0 || c >= nx) c = 0;  // lanes past a narrow lattice
  const int xm = c == 0 ? nx - 1 : c - 1, xp = c == nx - 1 ? 0 : c + 1;
  const int dir = (by & 1) ? -1 : 1;
  const int nit = Y1 - Y0 + 4;
  const int rfirst = dir > 0 ? Y0 - 2 : Y1 + 1;
  auto wrap = [&](int r) { return r < 0 ? r + ny : (r >= ny ? r - ny : r); };
  // the 18 pulled values and the node's phi history of row r, issued
  // together by every lane (loads complete in order, so a value loaded
  // after the next row's pull would make its use wait for that whole pull)
  auto pull = [&](int r, T* f, T* g, T& ph) {
    const int y = wrap(r), ym = wrap(r - 1), yp = wrap(r + 1);
    const int ys[9] = {y, y, ym, y, yp, ym, ym, yp, yp};
    const int xs[9] = {c, xm, c, xp, c, xm, xp, xp, xm};
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      f[a] = F[pix(nx, a, ys[a], xs[a])];
      g[a] = G[pix(nx, a, ys[a], xs[a])];
    }
    ph = PI[(long long)y * nx + c];
  };
  Gbl<T>* SK = (Gbl<T>*)sink;
  auto store = [&](int r, const T* f, const T* g, T ph) {
    const bool real = own && r >= Y0 && r < Y1;
    const long long rr = real ? r : 0;
    Gbl<T>* fo = real ? FO : SK;
    Gbl<T>* go = real ? GO : SK + 9 * (long long)nx;
    Gbl<T>* po = real ? PO : SK + 18 * (long long)nx;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
      fo[pix(nx, a, rr, c)] = f[a];
      go[pix(nx, a, rr, c)] = g[a];
    }
    po[rr * nx + c] = ph;
  };
  T f0[9], g0[9], f1[9], g1[9], p0, p1;
  pull(rfirst, f0, g0, p0);
  for (int it = 0; it < nit; it += 2) {
    const int r = rfirst + dir * it;
    pull(r + dir, f1, g1, p1);   // row r + 1 in flight while row r is stored
    store(r, f0, g0, p0);
    pull(r + 2 * dir, f0, g0, p0);
    store(r + dir, f1, g1, p1);
  }
}

}  // namespace

extern "C" {

// Streaming probes over `bytes` (a multiple of 16) on `stream`, with
// `blocks` blocks of 256 threads (grid-stride): kind 0 copies src to dst,
// 1 the same with non-temporal accesses, 2 reads src only (dst receives
// blocks x 256 x 16 bytes), 3 writes dst only.  Returns 0, -1 for an unknown
// kind, -2 when the launch fails.
int lbpc_probe_stream(int kind, const void* src, void* dst, size_t bytes,
                      int blocks, void* stream) {
  const long long n = (long long)(bytes / 16);
  hipStream_t s = (hipStream_t)stream;
  const u32x4* a = (const u32x4*)src;
  u32x4* b = (u32x4*)dst;
  switch (kind) {
    case 0: hipLaunchKernelGGL((k_copy<4, false>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    case 1: hipLaunchKernelGGL((k_copy<4, true>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    case 2: hipLaunchKernelGGL((k_read<4>), dim3(blocks), dim3(256), 0, s, a, b, n); break;
    case 3: hipLaunchKernelGGL((k_write<4>), dim3(blocks), dim3(256), 0, s, b, n); break;
    default: return -1;
  }
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

// One pull-stream pass of the step's access pattern over a periodic nx x ny
// lattice (nx, ny >= 16): fin/gin/fout/gout hold 9 nx ny values of
// elem_bytes (8 or 4) in [ny][9][nx] rows, phin/phout nx ny values of the
// same type, sink 19 nx values.  Block of bw (256 or 512) threads, strips of W <= bw - 4
// columns, runs of H rows.  Returns 0, -1 for unsupported arguments, -2 when
// the launch fails.
int lbpc_probe_pattern(const void* fin, const void* gin, void* fout,
                       void* gout, const void* phin, void* phout, void* sink,
                       int nx, int ny, int elem_bytes, int bw, int W, int H,
                       void* stream) {
  // rows up to 5 beyond a run are pulled (wrapped once): ny >= 16
  if (nx < 16 || ny < 16 || W < 1 || W > bw - 4 || H < 1) return -1;
  const int nbx = (nx + W - 1) / W, nby = (ny + H - 1) / H;
  const dim3 grid(nbx * nby);
  hipStream_t s = (hipStream_t)stream;
#define LBPC_PROBE(T, BW)                                                      \
  hipLaunchKernelGGL((k_pattern<T, BW>), grid, dim3(BW), 0, s, (const T*)fin,  \
                     (const T*)gin, (T*)fout, (T*)gout, (const T*)phin,        \
                     (T*)phout, (T*)sink, nx, ny, W, H, nbx)
  if (elem_bytes == 8 && bw == 512) LBPC_PROBE(double, 512);
  else if (elem_bytes == 8 && bw == 256) LBPC_PROBE(double, 256);
  else if (elem_bytes == 4 && bw == 512) LBPC_PROBE(float, 512);
  else if (elem_bytes == 4 && bw == 256) LBPC_PROBE(float, 256);
  else return -1;
#undef LBPC_PROBE
  return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // extern "C"
