// FFT passes of the 3-D real transforms (Sec. 3.1) and the fused tangent x pass.
//
//  * x pass: real rows <-> half-spectrum rows, two real rows packed per complex
//    pencil; the fused variant applies the degraded tangent g K : eps between the
//    inverse and the forward row transforms (the real-space factor of the linearised
//    equilibrium operator of eq. newton);
//  * y / z passes: complex pencils along a strided axis; a block stages a tile of TX
//    x-adjacent pencils in LDS so that every global access is contiguous along x.
// Every common axis length is compiled as its own kernel (all index arithmetic by
// constants); other 2^a 3^b lengths use the runtime-length kernel.
#include "kernels.h"
#include "fft.h"
#include "regfft.h"
#include <cmath>

namespace rvefft {

template <typename R>
__device__ __forceinline__ void load_twiddles(cplx<R>* tw_s, const cplx<R>* tw_g, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) tw_s[t] = tw_g[t];
}

// Half-spectrum bin k of a real row, read as a Hermitian row (imaginary parts of bin
// 0 and of the Nyquist bin dropped: they do not exist for a real row).
template <typename R>
__device__ __forceinline__ cplx<R> herm_bin(const cplx<R>* row, int k, int N) {
  const int NH = N / 2 + 1;
  if (k < NH) {
    cplx<R> v = row[k];
    if (k == 0 || (N % 2 == 0 && k == N / 2)) v.y = 0;
    return v;
  }
  cplx<R> v = row[N - k];
  v.y = -v.y;
  return v;
}

template <typename R, int NC>
__device__ __forceinline__ cplx<R>* row_fft(cplx<R>* A, cplx<R>* B, const cplx<R>* tw,
                                            const AxisPlan& pl, int P, bool inv) {
  if constexpr (NC > 0) return fft_rows_ct<R, NC>(A, B, tw, P, inv);
  else return fft_pencils<R, false>(A, B, tw, pl, P, 1, pl.n + 1, inv);
}

constexpr int kMaxRowPairs = 32;

// Per-pencil row bookkeeping of the x passes: pencil p of the block packs the rows
// r0 = 2(pair0+p) and r1 = r0+1 of the flattened (component, k, j) order.
struct RowPair {
  long long c0, rem0, c1, rem1;   // component and voxel row of each real row (-1: none)
};

__device__ __forceinline__ void row_pairs(RowPair* rp, int P, long long pair0, long long rows_per_comp,
                                          long long nrows) {
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const long long r0 = 2 * (pair0 + p), r1 = r0 + 1;
    RowPair q;
    q.c0 = (r0 < nrows) ? r0 / rows_per_comp : -1;
    q.rem0 = (r0 < nrows) ? r0 % rows_per_comp : 0;
    q.c1 = (r1 < nrows) ? r1 / rows_per_comp : -1;
    q.rem1 = (r1 < nrows) ? r1 % rows_per_comp : 0;
    rp[p] = q;
  }
}

// ---------------------------------------------------------------------------
// x pass, real -> half spectrum (optionally multiplying the input by g(phi)).
template <typename R, typename TI, int NC>
__global__ void __launch_bounds__(256)
k_x_r2c(const TI* __restrict__ in, long long in_cs, const double* __restrict__ phi, double kres,
        cplx<R>* __restrict__ out, long long out_cs, int ncomp, Grid g, AxisPlan pl,
        const cplx<R>* __restrict__ tw_g, int P) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ RowPair rp[kMaxRowPairs];
  const int N = NC > 0 ? NC : g.n1;
  const int NH = N / 2 + 1, pitch = N + 1;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long rows_per_comp = (long long)g.n2 * g.n3;
  row_pairs(rp, P, (long long)blockIdx.x * P, rows_per_comp, rows_per_comp * ncomp);
  __syncthreads();
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, i = t % N;
    const RowPair q = rp[p];
    R a = 0, b = 0;
    if (q.c0 >= 0) {
      const long long v = q.rem0 * N + i;
      double x = (double)in[q.c0 * in_cs + v];
      if (phi) { const double u = 1.0 - phi[v]; x *= u * u + kres; }
      a = (R)x;
    }
    if (q.c1 >= 0) {
      const long long v = q.rem1 * N + i;
      double x = (double)in[q.c1 * in_cs + v];
      if (phi) { const double u = 1.0 - phi[v]; x *= u * u + kres; }
      b = (R)x;
    }
    A[p * pitch + i] = cplx<R>{a, b};
  }
  __syncthreads();
  cplx<R>* Z = row_fft<R, NC>(A, B, tw, pl, P, false);
  for (int t = threadIdx.x; t < P * NH; t += blockDim.x) {
    const int p = t / NH, k = t % NH;
    const RowPair q = rp[p];
    if (q.c0 < 0) continue;
    const cplx<R> zk = Z[p * pitch + k];
    const cplx<R> zm = Z[p * pitch + ((N - k) % N)];
    // A_k = (Z_k + conj Z_-k)/2 ; B_k = (Z_k - conj Z_-k)/(2i)
    out[q.c0 * out_cs + q.rem0 * NH + k] = cplx<R>{R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    if (q.c1 >= 0)
      out[q.c1 * out_cs + q.rem1 * NH + k] =
          cplx<R>{R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
  }
}

// x pass, half spectrum -> real: out = scale * x (or out += scale * x).
template <typename R, typename TO, int NC>
__global__ void __launch_bounds__(256)
k_x_c2r(const cplx<R>* __restrict__ in, long long in_cs, TO* __restrict__ out, long long out_cs,
        int ncomp, double scale, int accumulate, Grid g, AxisPlan pl,
        const cplx<R>* __restrict__ tw_g, int P) {
  extern __shared__ unsigned char smem_raw[];
  __shared__ RowPair rp[kMaxRowPairs];
  const int N = NC > 0 ? NC : g.n1;
  const int NH = N / 2 + 1, pitch = N + 1;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long rows_per_comp = (long long)g.n2 * g.n3;
  row_pairs(rp, P, (long long)blockIdx.x * P, rows_per_comp, rows_per_comp * ncomp);
  __syncthreads();
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, k = t % N;
    const RowPair q = rp[p];
    cplx<R> a = {0, 0}, b = {0, 0};
    if (q.c0 >= 0) a = herm_bin(in + q.c0 * in_cs + q.rem0 * NH, k, N);
    if (q.c1 >= 0) b = herm_bin(in + q.c1 * in_cs + q.rem1 * NH, k, N);
    A[p * pitch + k] = cplx<R>{a.x - b.y, a.y + b.x};     // a + i b
  }
  __syncthreads();
  cplx<R>* Z = row_fft<R, NC>(A, B, tw, pl, P, true);
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, i = t % N;
    const RowPair q = rp[p];
    if (q.c0 < 0) continue;
    const cplx<R> z = Z[p * pitch + i];
    {
      TO* o = out + q.c0 * out_cs + q.rem0 * N + i;
      const double v = scale * (double)z.x;
      *o = accumulate ? (TO)((double)*o + v) : (TO)v;
    }
    if (q.c1 >= 0) {
      TO* o = out + q.c1 * out_cs + q.rem1 * N + i;
      const double v = scale * (double)z.y;
      *o = accumulate ? (TO)((double)*o + v) : (TO)v;
    }
  }
}

// Fused x pass of the equilibrium operator on 6 components (in place):
//   eps = F_x^-1{.}, sigma = scale * gK : eps (Mandel), out = F_x{sigma}.
// One block holds Q voxel rows; components (xx,yy), (zz,yz), (xz,xy) share pencils.
template <typename R, int NC>
__global__ void __launch_bounds__(256)
k_x_tangent(cplx<R>* __restrict__ data, long long cs, const R* __restrict__ gK, double scale,
            Grid g, AxisPlan pl, const cplx<R>* __restrict__ tw_g, int Q,
            const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  const int N = NC > 0 ? NC : g.n1;
  const int NH = N / 2 + 1, pitch = N + 1;
  const int P = 3 * Q;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long nrows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * Q;
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, k = t % N;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    cplx<R> a = {0, 0}, b = {0, 0};
    if (rem < nrows) {
      a = herm_bin(data + (2 * pair) * cs + rem * NH, k, N);
      b = herm_bin(data + (2 * pair + 1) * cs + rem * NH, k, N);
    }
    A[p * pitch + k] = cplx<R>{a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  cplx<R>* Z = row_fft<R, NC>(A, B, tw, pl, P, true);
  cplx<R>* W = (Z == A) ? B : A;
  const R s2 = (R)1.41421356237309504880;
  const R is2 = (R)0.70710678118654752440;
  for (int t = threadIdx.x; t < Q * N; t += blockDim.x) {
    const int q = t / N, i = t % N;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const long long v = rem * N + i;
    const cplx<R> z0 = Z[(3 * q + 0) * pitch + i];
    const cplx<R> z1 = Z[(3 * q + 1) * pitch + i];
    const cplx<R> z2 = Z[(3 * q + 2) * pitch + i];
    const R e[6] = {z0.x, z0.y, z1.x, s2 * z1.y, s2 * z2.x, s2 * z2.y};   // Mandel strain
    R s[6] = {0, 0, 0, 0, 0, 0};
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) {
        const R k = gK[(long long)idx * g.nvox + v];
        s[a] += k * e[b];
        if (b != a) s[b] += k * e[a];
        ++idx;
      }
    const R sc = (R)scale;
    W[(3 * q + 0) * pitch + i] = cplx<R>{sc * s[0], sc * s[1]};
    W[(3 * q + 1) * pitch + i] = cplx<R>{sc * s[2], sc * is2 * s[3]};
    W[(3 * q + 2) * pitch + i] = cplx<R>{sc * is2 * s[4], sc * is2 * s[5]};
  }
  __syncthreads();
  cplx<R>* other = (W == A) ? B : A;
  cplx<R>* Y = row_fft<R, NC>(W, other, tw, pl, P, false);
  for (int t = threadIdx.x; t < P * NH; t += blockDim.x) {
    const int p = t / NH, k = t % NH;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const cplx<R> zk = Y[p * pitch + k];
    const cplx<R> zm = Y[p * pitch + ((N - k) % N)];
    data[(2 * pair) * cs + rem * NH + k] = cplx<R>{R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    data[(2 * pair + 1) * cs + rem * NH + k] =
        cplx<R>{R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
  }
}

// y (axis 1) or z (axis 2) pass, in place on ncomp components.  Block = (tile of
// TX x-bins) x (index along the remaining axis); blockIdx.y = component.
template <typename R, int NC, int TXC>
__global__ void __launch_bounds__(256)
k_fft_strided(cplx<R>* __restrict__ data, long long cs, int axis, int inv, Grid g, AxisPlan pl,
              const cplx<R>* __restrict__ tw_g, int TXr, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  const int N = NC > 0 ? NC : pl.n;
  const int TX = TXC > 0 ? TXC : TXr;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + TX * N;
  load_twiddles(tw, tw_g, N);
  const int ntiles = (g.n1h + TX - 1) / TX;
  const int tile = blockIdx.x % ntiles;
  const int other = blockIdx.x / ntiles;
  const int kx0 = tile * TX;
  long long stride_n, base;
  if (axis == 1) { stride_n = g.n1h; base = (long long)other * g.n1h * g.n2; }
  else { stride_n = (long long)g.n1h * g.n2; base = (long long)other * g.n1h; }
  cplx<R>* d = data + (long long)blockIdx.y * cs + base + kx0;
  const int w = min(TX, g.n1h - kx0);
  for (int t = threadIdx.x; t < TX * N; t += blockDim.x) {
    const int n = t / TX, x = t % TX;
    A[n * TX + x] = (x < w) ? d[n * stride_n + x] : cplx<R>{0, 0};
  }
  __syncthreads();
  cplx<R>* Z;
  if constexpr (NC > 0 && TXC > 0) Z = fft_tiles_ct<R, NC, TXC>(A, B, tw, inv != 0);
  else Z = fft_pencils<R, true>(A, B, tw, pl, TX, TX, 1, inv != 0);
  for (int t = threadIdx.x; t < TX * N; t += blockDim.x) {
    const int n = t / TX, x = t % TX;
    if (x < w) d[n * stride_n + x] = Z[n * TX + x];
  }
}

// Strided pass with a compile-time length and tile, single LDS buffer.  When the x
// size is even and N1/2 is a multiple of TX, the tiles cover kx in [0, N1/2) exactly
// and every block carries one extra pencil slot that tile 0 uses for the Nyquist
// column kx = N1/2 (the other tiles leave it idle): no ragged tiles.
template <typename R, int NC, int TXC, bool NYQ>
__global__ void __launch_bounds__(256)
k_fft_strided_ip(cplx<R>* __restrict__ data, long long cs, int axis, int inv, Grid g,
                 const cplx<R>* __restrict__ tw_g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  constexpr int P = NYQ ? TXC + 1 : TXC;
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + NC;
  load_twiddles(tw, tw_g, NC);
  const int ntiles = NYQ ? (g.n1 / 2) / TXC : (g.n1h + TXC - 1) / TXC;
  const int tile = blockIdx.x % ntiles;
  const int other = blockIdx.x / ntiles;
  const int kx0 = tile * TXC;
  long long stride_n, base;
  if (axis == 1) { stride_n = g.n1h; base = (long long)other * g.n1h * g.n2; }
  else { stride_n = (long long)g.n1h * g.n2; base = (long long)other * g.n1h; }
  cplx<R>* d = data + (long long)blockIdx.y * cs + base;
  // column of pencil slot x, or -1 if idle
  auto col = [&](int x) -> int {
    if (x < TXC) {
      const int c = kx0 + x;
      return (c < g.n1h) ? c : -1;
    }
    return (tile == 0) ? g.n1 / 2 : -1;
  };
  for (int t = threadIdx.x; t < P * NC; t += 256) {
    const int n = t / P, x = t % P;
    const int c = col(x);
    A[n * P + x] = (c >= 0) ? d[n * stride_n + c] : cplx<R>{0, 0};
  }
  __syncthreads();
  ct_run_ip<R, NC, 0, 1, P, 1, P, true, 256>(A, tw, inv != 0);
  for (int t = threadIdx.x; t < P * NC; t += 256) {
    const int n = t / P, x = t % P;
    const int c = col(x);
    if (c >= 0) d[n * stride_n + c] = A[n * P + x];
  }
}

// Software-pipelined variant: a block transforms CPB components of its tile in turn;
// the global loads of the next component are issued before the current component's
// butterflies, so the memory system stays busy while the block computes.
template <typename R, int NC, int TXC, bool NYQ, int CPB>
__global__ void __launch_bounds__(256)
k_fft_strided_pipe(cplx<R>* __restrict__ data, long long cs, int axis, int inv, Grid g,
                   const cplx<R>* __restrict__ tw_g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  constexpr int P = NYQ ? TXC + 1 : TXC;
  constexpr int E = (P * NC + 255) / 256;
  extern __shared__ unsigned char smem_raw[];
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + NC;
  load_twiddles(tw, tw_g, NC);
  const int ntiles = NYQ ? (g.n1 / 2) / TXC : (g.n1h + TXC - 1) / TXC;
  const int tile = blockIdx.x % ntiles;
  const int other = blockIdx.x / ntiles;
  const int kx0 = tile * TXC;
  long long stride_n, base;
  if (axis == 1) { stride_n = g.n1h; base = (long long)other * g.n1h * g.n2; }
  else { stride_n = (long long)g.n1h * g.n2; base = (long long)other * g.n1h; }
  const cplx<R>* d0 = data + (long long)blockIdx.y * CPB * cs + base;
  long long goff[E];
#pragma unroll
  for (int e = 0; e < E; ++e) {
    const int t = threadIdx.x + e * 256;
    goff[e] = -1;
    if (t < P * NC) {
      const int n = t / P, x = t % P;
      int c;
      if (x < TXC) c = (kx0 + x < g.n1h) ? kx0 + x : -1;
      else c = (tile == 0) ? g.n1 / 2 : -1;
      if (c >= 0) goff[e] = n * stride_n + c;
    }
  }
  cplx<R> reg[E];
#pragma unroll
  for (int e = 0; e < E; ++e) reg[e] = (goff[e] >= 0) ? d0[goff[e]] : cplx<R>{0, 0};
  for (int cc = 0; cc < CPB; ++cc) {
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = threadIdx.x + e * 256;
      if (t < P * NC) A[t] = reg[e];          // layout [n][P]: t = n*P + x
    }
    __syncthreads();
    if (cc + 1 < CPB) {
      const cplx<R>* dn = d0 + (cc + 1) * cs;
#pragma unroll
      for (int e = 0; e < E; ++e) reg[e] = (goff[e] >= 0) ? dn[goff[e]] : cplx<R>{0, 0};
    }
    ct_run_ip<R, NC, 0, 1, P, 1, P, true, 256>(A, tw, inv != 0);
    cplx<R>* dc = data + ((long long)blockIdx.y * CPB + cc) * cs + base;
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int t = threadIdx.x + e * 256;
      if (goff[e] >= 0) dc[goff[e]] = A[t];
    }
    __syncthreads();
  }
}

// Fused tangent x pass with a compile-time row length and rows per block, single LDS
// buffer (in-place Stockham stages, fft.h): same arithmetic as k_x_tangent.
template <typename R, int N, int Q, int NT>
__global__ void __launch_bounds__(NT)
k_x_tangent_ip(cplx<R>* __restrict__ data, long long cs, const R* __restrict__ gK, double scale,
               Grid g, const cplx<R>* __restrict__ tw_g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  constexpr int NH = N / 2 + 1, PITCH = N + 1, P = 3 * Q;
  __shared__ cplx<R> tw[N];
  __shared__ cplx<R> A[P * PITCH];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const long long nrows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * Q;
  for (int t = threadIdx.x; t < P * N; t += NT) {
    const int p = t / N, k = t % N;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    cplx<R> a = {0, 0}, b = {0, 0};
    if (rem < nrows) {
      a = herm_bin(data + (2 * pair) * cs + rem * NH, k, N);
      b = herm_bin(data + (2 * pair + 1) * cs + rem * NH, k, N);
    }
    A[p * PITCH + k] = cplx<R>{a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  ct_run_ip<R, N, 0, 1, 1, PITCH, P, false, NT>(A, tw, true);
  const R s2 = (R)1.41421356237309504880;
  const R is2 = (R)0.70710678118654752440;
  const R sc = (R)scale;
  for (int t = threadIdx.x; t < Q * N; t += NT) {
    const int q = t / N, i = t % N;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const long long v = rem * N + i;
    const cplx<R> z0 = A[(3 * q + 0) * PITCH + i];
    const cplx<R> z1 = A[(3 * q + 1) * PITCH + i];
    const cplx<R> z2 = A[(3 * q + 2) * PITCH + i];
    const R e[6] = {z0.x, z0.y, z1.x, s2 * z1.y, s2 * z2.x, s2 * z2.y};
    R s[6] = {0, 0, 0, 0, 0, 0};
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) {
        const R k = gK[(long long)idx * g.nvox + v];
        s[a] += k * e[b];
        if (b != a) s[b] += k * e[a];
        ++idx;
      }
    A[(3 * q + 0) * PITCH + i] = cplx<R>{sc * s[0], sc * s[1]};
    A[(3 * q + 1) * PITCH + i] = cplx<R>{sc * s[2], sc * is2 * s[3]};
    A[(3 * q + 2) * PITCH + i] = cplx<R>{sc * is2 * s[4], sc * is2 * s[5]};
  }
  __syncthreads();
  ct_run_ip<R, N, 0, 1, 1, PITCH, P, false, NT>(A, tw, false);
  for (int t = threadIdx.x; t < P * NH; t += NT) {
    const int p = t / NH, k = t % NH;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const cplx<R> zk = A[p * PITCH + k];
    const cplx<R> zm = A[p * PITCH + ((N - k) % N)];
    data[(2 * pair) * cs + rem * NH + k] = cplx<R>{R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    data[(2 * pair + 1) * cs + rem * NH + k] =
        cplx<R>{R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
  }
}

// Constant twiddle tables of the register DFTs.
__constant__ double c_tw256[2 * 256];
__constant__ double c_tw192[2 * 192];

// Strided pass by the two-pass register FFT (regfft.h).  P = TX (+1 Nyquist slot, see
// k_fft_strided_ip) pencils of length N per block, LDS holds one transposition buffer.
template <typename R, int N, int TX, bool NYQ, bool INV, int NT>
__global__ void __launch_bounds__(NT)
k_fft_strided_reg(cplx<R>* __restrict__ data, long long cs, int axis, Grid g,
                  const cplx<R>* __restrict__ tw_g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  constexpr int P = NYQ ? TX + 1 : TX;
  constexpr int Na = TwoPass<N>::Na, Nb = TwoPass<N>::Nb;
  constexpr int PITCH = N + 1;
  __shared__ cplx<R> A[P * PITCH];
  __shared__ cplx<R> tw[N];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const int ntiles = NYQ ? (g.n1 / 2) / TX : (g.n1h + TX - 1) / TX;
  const int tile = blockIdx.x % ntiles;
  const int other = blockIdx.x / ntiles;
  const int kx0 = tile * TX;
  long long stride_n, base;
  if (axis == 1) { stride_n = g.n1h; base = (long long)other * g.n1h * g.n2; }
  else { stride_n = (long long)g.n1h * g.n2; base = (long long)other * g.n1h; }
  cplx<R>* d = data + (long long)blockIdx.y * cs + base;
  auto col = [&](int x) -> int {
    if (x < TX) return (kx0 + x < g.n1h) ? kx0 + x : -1;
    return (tile == 0) ? g.n1 / 2 : -1;
  };
  __syncthreads();
  for (int t = threadIdx.x; t < P * Nb; t += NT) {
    const int x = t % P, n1 = t / P;
    const int c = col(x);
    cplx<R> v[Na];
#pragma unroll
    for (int m = 0; m < Na; ++m) v[m] = (c >= 0) ? d[(long long)(n1 + Nb * m) * stride_n + c] : cplx<R>{0, 0};
    reg_dft<R, Na, INV>(v);
#pragma unroll
    for (int k2 = 0; k2 < Na; ++k2) {
      cplx<R> w = tw[n1 * k2];
      if (INV) w.y = -w.y;
      A[x * PITCH + n1 + Nb * k2] = (k2 == 0) ? v[k2] : cmul(v[k2], w);
    }
  }
  __syncthreads();
  for (int t = threadIdx.x; t < P * Na; t += NT) {
    const int x = t % P, k2 = t / P;
    const int c = col(x);
    cplx<R> v[Nb];
#pragma unroll
    for (int n1 = 0; n1 < Nb; ++n1) v[n1] = A[x * PITCH + n1 + Nb * k2];
    reg_dft<R, Nb, INV>(v);
    if (c >= 0) {
#pragma unroll
      for (int k1 = 0; k1 < Nb; ++k1) d[(long long)(k2 + Na * k1) * stride_n + c] = v[k1];
    }
  }
}

// ---------------------------------------------------------------------------
// z passes fused with the pointwise operators at the two ends of the momentum
// operator (Sec. 3.1, eqs. fdef and momentum): the inverse pass forms the strain
// spectrum sym(i xi~ (x) p) of the updated CG direction while it loads, the forward
// pass contracts the stress spectrum with -i xi~ while it stores, so neither spectrum
// makes an extra trip through HBM.  A work unit is a tile of x-bins at one ky; each
// block takes one component of one unit.  When the units come in multiples of 8, the
// blocks of one unit are numbered 8 apart, so they are dispatched to the same XCD one
// after the other and meet the operands they share in its L2.
__device__ __forceinline__ void unit_comp(int nunits, int ncomp, int& u, int& c) {
  const int bid = blockIdx.x;
  if ((nunits & 7) == 0) {
    const int x = bid & 7, s = bid >> 3;
    c = s % ncomp;
    u = (s / ncomp) * 8 + x;
  } else {
    c = bid % ncomp;
    u = bid / ncomp;
  }
}

// i s a for real s
template <typename R>
__device__ __forceinline__ cplx<R> imul(R s, cplx<R> a) { return cplx<R>{-s * a.y, s * a.x}; }

// Split N = Na x Nb of the fused z passes: a short first pass, so that the several
// operands each first-pass item loads stay in registers together.
template <int N> struct ZSplit;
template <> struct ZSplit<16> { static constexpr int Na = 4, Nb = 4; };
template <> struct ZSplit<32> { static constexpr int Na = 4, Nb = 8; };
template <> struct ZSplit<48> { static constexpr int Na = 3, Nb = 16; };
template <> struct ZSplit<64> { static constexpr int Na = 8, Nb = 8; };
template <> struct ZSplit<96> { static constexpr int Na = 6, Nb = 16; };
template <> struct ZSplit<128> { static constexpr int Na = 8, Nb = 16; };
template <> struct ZSplit<256> { static constexpr int Na = 16, Nb = 16; };

// xi~ of the block's x columns, its ky and every kz, in LDS (no divisions in the loops)
template <typename R, int N, int P, int NT>
__device__ __forceinline__ void z_freqs(const Grid& g, int kx0, int tile, int TX, int ky,
                                        R* txs, R* tzs, R& ty) {
  for (int t = threadIdx.x; t < N; t += NT) tzs[t] = (R)freq(t, g.n3, g.L3, true);
  for (int t = threadIdx.x; t < P; t += NT) {
    const int cx = (t < TX) ? kx0 + t : (tile == 0 ? g.n1 / 2 : -1);
    txs[t] = cx >= 0 ? (R)freq(cx, g.n1, g.L1, true) : R(0);
  }
  ty = (R)freq(ky, g.n2, g.L2, true);
}

// p_new = z + (sc[ia]/sc[ib]) p_old, then component c of e = sym(i xi~ (x) p_new) and its
// inverse DFT along z.  The blocks of the diagonal components store p_new.
template <typename R, int N, int TX, int NT>
__global__ void __launch_bounds__(NT)
k_zgrad_inv(const cplx<R>* __restrict__ zv, const cplx<R>* __restrict__ pold,
            cplx<R>* __restrict__ pnew, long long cs, const double* __restrict__ sc, int ia,
            int ib, cplx<R>* __restrict__ e, Grid g, const cplx<R>* __restrict__ tw_g,
            const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  constexpr int P = TX + 1;                       // the Nyquist column rides in tile 0
  constexpr int Na = ZSplit<N>::Na, Nb = ZSplit<N>::Nb;
  constexpr int PITCH = N + 1;
  __shared__ cplx<R> A[P * PITCH];
  __shared__ cplx<R> tw[N];
  __shared__ R tzs[N], txs[P];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const int ntiles = (g.n1 / 2) / TX;
  int u, c;
  unit_comp(ntiles * g.n2, 6, u, c);
  const int tile = u % ntiles, ky = u / ntiles;
  const int kx0 = tile * TX;
  const long long stride_n = (long long)g.n1h * g.n2;
  const long long base = (long long)ky * g.n1h;
  R ty;
  z_freqs<R, N, P, NT>(g, kx0, tile, TX, ky, txs, tzs, ty);
  // component c = (a, b): xx, yy, zz, yz, xz, xy
  const int ca = (c < 3) ? c : (c == 3 ? 1 : 0);
  const int cb = (c < 3) ? c : (c == 5 ? 1 : 2);
  const double be = sc[ia] / sc[ib];
  auto col = [&](int x) -> int {
    if (x < TX) return kx0 + x;
    return (tile == 0) ? g.n1 / 2 : -1;
  };
  auto upd = [&](cplx<R> zz, cplx<R> pp) -> cplx<R> {
    return cplx<R>{(R)((double)zz.x + be * (double)pp.x), (R)((double)zz.y + be * (double)pp.y)};
  };
  __syncthreads();
  for (int t = threadIdx.x; t < P * Nb; t += NT) {
    const int x = t % P, n1 = t / P;
    const int cx = col(x);
    cplx<R> v[Na];
    if (cx >= 0) {
      const R tx = txs[x];
      const long long i0 = base + (long long)n1 * stride_n + cx;
      const long long sm = (long long)Nb * stride_n;
      cplx<R> za[Na], pa[Na];
#pragma unroll
      for (int m = 0; m < Na; ++m) {
        za[m] = zv[ca * cs + i0 + m * sm];
        pa[m] = pold[ca * cs + i0 + m * sm];
      }
#pragma unroll
      for (int m = 0; m < Na; ++m) v[m] = upd(za[m], pa[m]);     // p_new_a
      if (c < 3) {
#pragma unroll
        for (int m = 0; m < Na; ++m) {
          pnew[ca * cs + i0 + m * sm] = v[m];
          const R ta = (ca == 0) ? tx : (ca == 1 ? ty : tzs[n1 + Nb * m]);
          v[m] = imul(ta, v[m]);
        }
      } else {
        cplx<R> zb[Na], pb[Na];
#pragma unroll
        for (int m = 0; m < Na; ++m) {
          zb[m] = zv[cb * cs + i0 + m * sm];
          pb[m] = pold[cb * cs + i0 + m * sm];
        }
#pragma unroll
        for (int m = 0; m < Na; ++m) {
          const R tz = tzs[n1 + Nb * m];
          const R ta = (ca == 0) ? tx : ty;                  // off the diagonal a < b, a < 2
          const R tb = (cb == 1) ? ty : tz;
          const cplx<R> nb = upd(zb[m], pb[m]);
          v[m] = cscale(cadd(imul(ta, nb), imul(tb, v[m])), R(0.5));
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < Na; ++m) v[m] = cplx<R>{0, 0};
    }
    reg_dft<R, Na, true>(v);
#pragma unroll
    for (int k2 = 0; k2 < Na; ++k2) {
      cplx<R> w = tw[n1 * k2];
      w.y = -w.y;
      A[x * PITCH + n1 + Nb * k2] = (k2 == 0) ? v[k2] : cmul(v[k2], w);
    }
  }
  __syncthreads();
  cplx<R>* d = e + (long long)c * cs + base;
  for (int t = threadIdx.x; t < P * Na; t += NT) {
    const int x = t % P, k2 = t / P;
    const int cx = col(x);
    cplx<R> v[Nb];
#pragma unroll
    for (int n1 = 0; n1 < Nb; ++n1) v[n1] = A[x * PITCH + n1 + Nb * k2];
    reg_dft<R, Nb, true>(v);
    if (cx >= 0) {
#pragma unroll
      for (int k1 = 0; k1 < Nb; ++k1) d[(long long)(k2 + Na * k1) * stride_n + cx] = v[k1];
    }
  }
}

// Component i of q = -i xi~ . F_z{s} and the block partial of the Parseval-weighted
// <p, q>, in two rounds: xi~_z F_z{s_iz} first (its result waits in LDS), then
// F_z{xi~_x s_ix + xi~_y s_iy}, whose x and y factors are constant along z.
template <typename R, int N, int TX, int NT>
__global__ void __launch_bounds__(NT)
k_zdiv_fwd(const cplx<R>* __restrict__ s, cplx<R>* __restrict__ q, const cplx<R>* __restrict__ pv,
           long long cs, Grid g, const cplx<R>* __restrict__ tw_g, double* __restrict__ partial,
           const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  constexpr int P = TX + 1;
  constexpr int Na = ZSplit<N>::Na, Nb = ZSplit<N>::Nb;
  constexpr int PITCH = N + 1;
  __shared__ cplx<R> A[P * PITCH];
  __shared__ cplx<R> D[P * N];
  __shared__ cplx<R> tw[N];
  __shared__ R tzs[N], txs[P];
  __shared__ double red[NT / 64];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const int ntiles = (g.n1 / 2) / TX;
  int u, i;
  unit_comp(ntiles * g.n2, 3, u, i);
  const int tile = u % ntiles, ky = u / ntiles;
  const int kx0 = tile * TX;
  const long long stride_n = (long long)g.n1h * g.n2;
  const long long base = (long long)ky * g.n1h;
  R ty;
  z_freqs<R, N, P, NT>(g, kx0, tile, TX, ky, txs, tzs, ty);
  // s_ix, s_iy, s_iz among xx, yy, zz, yz, xz, xy
  const int sx = (i == 0) ? 0 : (i == 1 ? 5 : 4);
  const int sy = (i == 0) ? 5 : (i == 1 ? 1 : 3);
  const int sz = (i == 0) ? 4 : (i == 1 ? 3 : 2);
  auto col = [&](int x) -> int {
    if (x < TX) return kx0 + x;
    return (tile == 0) ? g.n1 / 2 : -1;
  };
  double acc = 0.0;
  __syncthreads();
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const bool zr = (round == 0);                               // the xi~_z round
    for (int t = threadIdx.x; t < P * Nb; t += NT) {
      const int x = t % P, n1 = t / P;
      const int cx = col(x);
      cplx<R> v[Na];
      if (cx >= 0) {
        const long long i0 = base + (long long)n1 * stride_n + cx;
        const long long sm = (long long)Nb * stride_n;
        if (zr) {
#pragma unroll
          for (int m = 0; m < Na; ++m) v[m] = s[sz * cs + i0 + m * sm];
        } else {
          const R tx = txs[x];
          cplx<R> a[Na], b[Na];
#pragma unroll
          for (int m = 0; m < Na; ++m) {
            a[m] = s[sx * cs + i0 + m * sm];
            b[m] = s[sy * cs + i0 + m * sm];
          }
#pragma unroll
          for (int m = 0; m < Na; ++m) v[m] = cadd(cscale(a[m], tx), cscale(b[m], ty));
        }
      } else {
#pragma unroll
        for (int m = 0; m < Na; ++m) v[m] = cplx<R>{0, 0};
      }
      reg_dft<R, Na, false>(v);
#pragma unroll
      for (int k2 = 0; k2 < Na; ++k2)
        A[x * PITCH + n1 + Nb * k2] = (k2 == 0) ? v[k2] : cmul(v[k2], tw[n1 * k2]);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P * Na; t += NT) {
      const int x = t % P, k2 = t / P;
      const int cx = col(x);
      cplx<R> v[Nb];
#pragma unroll
      for (int n1 = 0; n1 < Nb; ++n1) v[n1] = A[x * PITCH + n1 + Nb * k2];
      reg_dft<R, Nb, false>(v);
      if (cx < 0) continue;
      if (zr) {
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) v[k1] = cscale(v[k1], tzs[k2 + Na * k1]);
      }
      if (round == 0) {
        // D is private to the thread that owns item (x, k2) in both rounds
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) D[x * N + k2 + Na * k1] = v[k1];
      } else {
        const long long i0 = (long long)i * cs + base + (long long)k2 * stride_n + cx;
        const long long sk = (long long)Na * stride_n;
        cplx<R> pp[Nb];
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) pp[k1] = pv[i0 + k1 * sk];
        double dot = 0.0;
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) {
          const cplx<R> dd = cadd(v[k1], D[x * N + k2 + Na * k1]);
          const cplx<R> qq = {dd.y, -dd.x};                 // -i d
          q[i0 + k1 * sk] = qq;
          dot += (double)pp[k1].x * (double)qq.x + (double)pp[k1].y * (double)qq.y;
        }
        acc += parseval_w(cx, g.n1) * dot;
      }
    }
    __syncthreads();
  }
  block_partial_sum(acc, partial, red);
}

void upload_reg_twiddles(hipStream_t st) {
  static double t256[512], t192[384];
  for (int k = 0; k < 256; ++k) {
    t256[2 * k] = std::cos(-2.0 * M_PI * k / 256.0);
    t256[2 * k + 1] = std::sin(-2.0 * M_PI * k / 256.0);
  }
  for (int k = 0; k < 192; ++k) {
    t192[2 * k] = std::cos(-2.0 * M_PI * k / 192.0);
    t192[2 * k + 1] = std::sin(-2.0 * M_PI * k / 192.0);
  }
  (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tw256), t256, sizeof(t256), 0, hipMemcpyHostToDevice, st);
  (void)hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tw192), t192, sizeof(t192), 0, hipMemcpyHostToDevice, st);
  (void)hipStreamSynchronize(st);
}

// ---------------------------------------------------------------------------
// Host launchers.
static constexpr size_t kLdsBudget = 64 * 1024;

static size_t xpass_smem(int n1, int P, size_t csz) {
  return ((size_t)n1 + (size_t)P * (n1 + 1) * 2) * csz;
}

template <typename R>
static int pick_rows(int n1, int maxP) {
  int P = maxP;
  while (P > 1 && xpass_smem(n1, P, sizeof(cplx<R>)) > kLdsBudget) P /= 2;
  return P;
}

// Calls F.template operator()<NC>() with the compile-time length of n (0 if none).
template <typename F>
static void with_length(int n, F&& f) {
  switch (n) {
    case 16: f.template operator()<16>(); break;
    case 32: f.template operator()<32>(); break;
    case 48: f.template operator()<48>(); break;
    case 64: f.template operator()<64>(); break;
    case 96: f.template operator()<96>(); break;
    case 128: f.template operator()<128>(); break;
    case 256: f.template operator()<256>(); break;
    default: f.template operator()<0>(); break;
  }
}

template <typename R>
void launch_x_r2c(const Plans& p, const void* in, bool in_f64, long long in_cs, const double* phi,
                  double kres, cplx<R>* out, long long out_cs, int ncomp, hipStream_t st) {
  const Grid& g = p.g;
  const int P = pick_rows<R>(g.n1, 16);
  const long long pairs = ((long long)g.n2 * g.n3 * ncomp + 1) / 2;
  const int nblk = (int)((pairs + P - 1) / P);
  const size_t sm = xpass_smem(g.n1, P, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  with_length(g.n1, [&]<int NC>() {
    if (in_f64)
      hipLaunchKernelGGL((k_x_r2c<R, double, NC>), dim3(nblk), dim3(256), sm, st,
                         (const double*)in, in_cs, phi, kres, out, out_cs, ncomp, g, p.ax[0], tw, P);
    else
      hipLaunchKernelGGL((k_x_r2c<R, float, NC>), dim3(nblk), dim3(256), sm, st, (const float*)in,
                         in_cs, phi, kres, out, out_cs, ncomp, g, p.ax[0], tw, P);
  });
}

template <typename R>
void launch_x_c2r(const Plans& p, const cplx<R>* in, long long in_cs, void* out, bool out_f64,
                  long long out_cs, int ncomp, double scale, int accumulate, hipStream_t st) {
  const Grid& g = p.g;
  const int P = pick_rows<R>(g.n1, 16);
  const long long pairs = ((long long)g.n2 * g.n3 * ncomp + 1) / 2;
  const int nblk = (int)((pairs + P - 1) / P);
  const size_t sm = xpass_smem(g.n1, P, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  with_length(g.n1, [&]<int NC>() {
    if (out_f64)
      hipLaunchKernelGGL((k_x_c2r<R, double, NC>), dim3(nblk), dim3(256), sm, st, in, in_cs,
                         (double*)out, out_cs, ncomp, scale, accumulate, g, p.ax[0], tw, P);
    else
      hipLaunchKernelGGL((k_x_c2r<R, float, NC>), dim3(nblk), dim3(256), sm, st, in, in_cs,
                         (float*)out, out_cs, ncomp, scale, accumulate, g, p.ax[0], tw, P);
  });
}

template <typename R>
void launch_x_tangent(const Plans& p, cplx<R>* data, long long cs, const R* gK, double scale,
                      hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  int Q = 8;
  while (Q > 1 && xpass_smem(g.n1, 3 * Q, sizeof(cplx<R>)) > kLdsBudget) Q /= 2;
  const long long rows = (long long)g.n2 * g.n3;
  const int nblk = (int)((rows + Q - 1) / Q);
  const size_t sm = xpass_smem(g.n1, 3 * Q, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  bool done = false;
  with_length(g.n1, [&]<int NC>() {
    if constexpr (NC > 0) {
      // rows per block and block size, from sweeps at 128^3 (FP64 and FP32)
      auto go = [&]<int QI, int NT>() {
        constexpr size_t lds = ((size_t)NC + 3 * QI * (NC + 1)) * sizeof(cplx<R>);
        if constexpr (lds <= 64 * 1024) {
          const int nb = (int)((rows + QI - 1) / QI);
          hipLaunchKernelGGL((k_x_tangent_ip<R, NC, QI, NT>), dim3(nb), dim3(NT), 0, st, data, cs,
                             gK, scale, g, tw, stop);
          done = true;
        }
      };
      if constexpr (NC <= 64) go.template operator()<8, 256>();
      else go.template operator()<1, 128>();
    }
  });
  if (done) return;
  hipLaunchKernelGGL((k_x_tangent<R, 0>), dim3(nblk), dim3(256), sm, st, data, cs, gK, scale, g,
                     p.ax[0], tw, Q, stop);
}

template <typename R, int NC, int TX, int CPB>
static bool launch_strided_pipe(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis,
                                bool inv, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  if (ncomp % CPB) return false;
  const bool nyq = (g.n1 % 2 == 0) && ((g.n1 / 2) % TX == 0);
  const int P = nyq ? TX + 1 : TX;
  const size_t sm = (size_t)(NC + P * NC) * sizeof(cplx<R>);
  if (sm > kLdsBudget) return false;
  const int ntiles = nyq ? (g.n1 / 2) / TX : (g.n1h + TX - 1) / TX;
  const int others = (axis == 1) ? g.n3 : g.n2;
  const dim3 grid(ntiles * others, ncomp / CPB);
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(axis, sizeof(R) == 8);
  if (nyq)
    hipLaunchKernelGGL((k_fft_strided_pipe<R, NC, TX, true, CPB>), grid, dim3(256), sm, st, data,
                       cs, axis, inv ? 1 : 0, g, tw, stop);
  else
    hipLaunchKernelGGL((k_fft_strided_pipe<R, NC, TX, false, CPB>), grid, dim3(256), sm, st, data,
                       cs, axis, inv ? 1 : 0, g, tw, stop);
  return true;
}

template <typename R, int NC, int TX>
static bool launch_strided_ip(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis,
                              bool inv, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  const bool nyq = (g.n1 % 2 == 0) && ((g.n1 / 2) % TX == 0);
  const int P = nyq ? TX + 1 : TX;
  const size_t sm = (size_t)(NC + P * NC) * sizeof(cplx<R>);
  if (sm > kLdsBudget) return false;
  const int ntiles = nyq ? (g.n1 / 2) / TX : (g.n1h + TX - 1) / TX;
  const int others = (axis == 1) ? g.n3 : g.n2;
  const dim3 grid(ntiles * others, ncomp);
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(axis, sizeof(R) == 8);
  if (nyq)
    hipLaunchKernelGGL((k_fft_strided_ip<R, NC, TX, true>), grid, dim3(256), sm, st, data, cs, axis,
                       inv ? 1 : 0, g, tw, stop);
  else
    hipLaunchKernelGGL((k_fft_strided_ip<R, NC, TX, false>), grid, dim3(256), sm, st, data, cs,
                       axis, inv ? 1 : 0, g, tw, stop);
  return true;
}

template <typename R, int N, int TX, bool NYQ>
static void launch_reg_tx(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis,
                          bool inv, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  constexpr int P = NYQ ? TX + 1 : TX;
  constexpr int items = P * TwoPass<N>::Nb;
  constexpr int NT = ((items + 63) / 64) * 64 > 1024 ? 1024 : ((items + 63) / 64) * 64;
  const int ntiles = NYQ ? (g.n1 / 2) / TX : (g.n1h + TX - 1) / TX;
  const int others = (axis == 1) ? g.n3 : g.n2;
  const dim3 grid(ntiles * others, ncomp);
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(axis, sizeof(R) == 8);
  if (inv)
    hipLaunchKernelGGL((k_fft_strided_reg<R, N, TX, NYQ, true, NT>), grid, dim3(NT), 0, st, data,
                       cs, axis, g, tw, stop);
  else
    hipLaunchKernelGGL((k_fft_strided_reg<R, N, TX, NYQ, false, NT>), grid, dim3(NT), 0, st, data,
                       cs, axis, g, tw, stop);
}

// LDS bytes of k_fft_strided_reg
template <typename R>
constexpr size_t reg_lds(int N, int P) { return ((size_t)P * (N + 1) + N) * sizeof(cplx<R>); }
static constexpr size_t kRegLdsMax = 80 * 1024;

template <typename R, int N>
static bool launch_strided_reg(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis,
                               bool inv, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  const bool even = (g.n1 % 2 == 0);
  const int half = g.n1 / 2;
  if (even && half % 32 == 0 && reg_lds<R>(N, 33) <= kRegLdsMax)
    launch_reg_tx<R, N, 32, true>(p, data, cs, ncomp, axis, inv, st, stop);
  else if (even && half % 16 == 0 && reg_lds<R>(N, 17) <= kRegLdsMax)
    launch_reg_tx<R, N, 16, true>(p, data, cs, ncomp, axis, inv, st, stop);
  else if (even && half % 8 == 0 && reg_lds<R>(N, 9) <= kRegLdsMax)
    launch_reg_tx<R, N, 8, true>(p, data, cs, ncomp, axis, inv, st, stop);
  else if (reg_lds<R>(N, 16) <= kRegLdsMax)
    launch_reg_tx<R, N, 16, false>(p, data, cs, ncomp, axis, inv, st, stop);
  else
    return false;
  return true;
}

template <typename R>
void launch_fft_yz(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis, bool inv,
                   hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  const AxisPlan& pl = p.ax[axis];
  const int N = pl.n;
  bool done = false;
  with_length(N, [&]<int NC>() {
    if constexpr (NC > 0) {
      done = launch_strided_reg<R, NC>(p, data, cs, ncomp, axis, inv, st, stop) ||
             launch_strided_pipe<R, NC, 8, 3>(p, data, cs, ncomp, axis, inv, st, stop) ||
             launch_strided_ip<R, NC, 16>(p, data, cs, ncomp, axis, inv, st, stop) ||
             launch_strided_ip<R, NC, 8>(p, data, cs, ncomp, axis, inv, st, stop);
    }
  });
  if (done) return;
  int TX = 16;
  while (TX > 1 && ((size_t)N + 2 * (size_t)TX * N) * sizeof(cplx<R>) > kLdsBudget) TX /= 2;
  const int ntiles = (g.n1h + TX - 1) / TX;
  const int others = (axis == 1) ? g.n3 : g.n2;
  const size_t sm = ((size_t)N + 2 * (size_t)TX * N) * sizeof(cplx<R>);
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(axis, sizeof(R) == 8);
  const dim3 grid(ntiles * others, ncomp);
  hipLaunchKernelGGL((k_fft_strided<R, 0, 0>), grid, dim3(256), sm, st, data, cs, axis,
                     inv ? 1 : 0, g, pl, tw, TX, stop);
}

// LDS bytes of the fused z kernels
template <typename R>
constexpr size_t zgrad_lds(int N, int P) {
  return ((size_t)P * (N + 1) + N) * sizeof(cplx<R>) + (size_t)(N + P) * sizeof(R);
}
template <typename R>
constexpr size_t zdiv_lds(int N, int P) {
  return ((size_t)P * (N + 1) + (size_t)P * N + N) * sizeof(cplx<R>) +
         (size_t)(N + P) * sizeof(R) + 16 * sizeof(double);
}

// Largest x tile (32, 16 or 8 bins plus the Nyquist column) whose LDS fits; 0 if the
// grid has no fused z pass (odd n1, or n3 without a register DFT).
template <typename R, int N>
static int fused_tile(const Grid& g, bool div) {
  if (g.n1 % 2 != 0 || g.n3 != N) return 0;
  const int half = g.n1 / 2;
  for (int TX : {32, 16, 8}) {
    const size_t lds = div ? zdiv_lds<R>(N, TX + 1) : zgrad_lds<R>(N, TX + 1);
    if (half % TX == 0 && lds <= kRegLdsMax) return TX;
  }
  return 0;
}

template <int NT_ITEMS>
constexpr int threads_for() {
  return ((NT_ITEMS + 63) / 64) * 64 > 1024 ? 1024 : ((NT_ITEMS + 63) / 64) * 64;
}

template <typename R>
bool fused_z_available(const Plans& p) {
  bool ok = false;
  with_length(p.g.n3, [&]<int NC>() {
    if constexpr (NC > 0) ok = fused_tile<R, NC>(p.g, false) > 0 && fused_tile<R, NC>(p.g, true) > 0;
  });
  return ok;
}

template <typename R>
void launch_zgrad_inv(const Plans& p, const cplx<R>* z, const cplx<R>* pold, cplx<R>* pnew,
                      long long cs, const double* sc, int ia, int ib, cplx<R>* e, hipStream_t st,
                      const double* stop) {
  const Grid& g = p.g;
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(2, sizeof(R) == 8);
  with_length(g.n3, [&]<int NC>() {
    if constexpr (NC > 0) {
      const int TX = fused_tile<R, NC>(g, false);
      auto go = [&]<int T>() {
        constexpr int NT = threads_for<(T + 1) * ZSplit<NC>::Nb>();
        const int nblk = (g.n1 / 2 / T) * g.n2 * 6;
        hipLaunchKernelGGL((k_zgrad_inv<R, NC, T, NT>), dim3(nblk), dim3(NT), 0, st, z, pold,
                           pnew, cs, sc, ia, ib, e, g, tw, stop);
      };
      if (TX == 32) {
        if constexpr (zgrad_lds<R>(NC, 33) <= kRegLdsMax) go.template operator()<32>();
      } else if (TX == 16) {
        if constexpr (zgrad_lds<R>(NC, 17) <= kRegLdsMax) go.template operator()<16>();
      } else if (TX == 8) {
        if constexpr (zgrad_lds<R>(NC, 9) <= kRegLdsMax) go.template operator()<8>();
      }
    }
  });
}

template <typename R>
int launch_zdiv_fwd(const Plans& p, const cplx<R>* s, cplx<R>* q, const cplx<R>* pv, long long cs,
                    double* partial, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(2, sizeof(R) == 8);
  int nblk = 0;
  with_length(g.n3, [&]<int NC>() {
    if constexpr (NC > 0) {
      const int TX = fused_tile<R, NC>(g, true);
      auto go = [&]<int T>() {
        constexpr int NT = threads_for<(T + 1) * ZSplit<NC>::Nb>();
        nblk = (g.n1 / 2 / T) * g.n2 * 3;
        hipLaunchKernelGGL((k_zdiv_fwd<R, NC, T, NT>), dim3(nblk), dim3(NT), 0, st, s, q, pv, cs,
                           g, tw, partial, stop);
      };
      if (TX == 32) {
        if constexpr (zdiv_lds<R>(NC, 33) <= kRegLdsMax) go.template operator()<32>();
      } else if (TX == 16) {
        if constexpr (zdiv_lds<R>(NC, 17) <= kRegLdsMax) go.template operator()<16>();
      } else if (TX == 8) {
        if constexpr (zdiv_lds<R>(NC, 9) <= kRegLdsMax) go.template operator()<8>();
      }
    }
  });
  return nblk;
}

#define RVE_PASS_INST(R)                                                                         \
  template void launch_x_r2c<R>(const Plans&, const void*, bool, long long, const double*, double, \
                                cplx<R>*, long long, int, hipStream_t);                          \
  template void launch_x_c2r<R>(const Plans&, const cplx<R>*, long long, void*, bool, long long,  \
                                int, double, int, hipStream_t);                                  \
  template void launch_x_tangent<R>(const Plans&, cplx<R>*, long long, const R*, double,          \
                                    hipStream_t, const double*);                                 \
  template void launch_fft_yz<R>(const Plans&, cplx<R>*, long long, int, int, bool, hipStream_t,  \
                                 const double*);                                                 \
  template bool fused_z_available<R>(const Plans&);                                              \
  template void launch_zgrad_inv<R>(const Plans&, const cplx<R>*, const cplx<R>*, cplx<R>*,       \
                                    long long, const double*, int, int, cplx<R>*, hipStream_t,   \
                                    const double*);                                              \
  template int launch_zdiv_fwd<R>(const Plans&, const cplx<R>*, cplx<R>*, const cplx<R>*,         \
                                  long long, double*, hipStream_t, const double*);

RVE_PASS_INST(double)
RVE_PASS_INST(float)

}  // namespace rvefft
