// Strided FFT passes of the 3-D real transforms (Sec. 3.1): complex pencils along y or
// z; a block stages a tile of TX x-adjacent pencils in LDS so that every global access
// is contiguous along x.  Every common axis length is compiled as its own kernel (all
// index arithmetic by constants); other 2^a 3^b lengths use the runtime-length kernel.
// The x passes are in xpass.hip, the z passes fused with the operator's end points in
// zfused.hip.
#include "passutil.h"
#include <cmath>

namespace rvefft {

// y (axis 1) or z (axis 2) pass, in place on ncomp components.  Block = (tile of
// TX x-bins) x (index along the remaining axis); blockIdx.y = component.
template <typename R, int NC, int TXC>
__global__ void __launch_bounds__(256)
k_fft_strided(cplx<R>* __restrict__ data, long long cs, int axis, int inv, Grid g, AxisPlan pl,
              const cplx<R>* __restrict__ tw_g, int TXr, const double* __restrict__ stop) {
  {
    const long long d = slot_delta(g);
    data = at_slot(data, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
  }
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
  {
    const long long d = slot_delta(g);
    data = at_slot(data, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
  }
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
  {
    const long long d = slot_delta(g);
    data = at_slot(data, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
  }
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


// Strided pass by the two-pass register FFT (regfft.h).  P = TX (+1 Nyquist slot, see
// k_fft_strided_ip) pencils of length N per block, LDS holds one transposition buffer.
template <typename R, int N, int TX, bool NYQ, bool INV, int NT>
__global__ void __launch_bounds__(NT)
k_fft_strided_reg(cplx<R>* __restrict__ data, long long cs, int axis, Grid g,
                  const cplx<R>* __restrict__ tw_g, const double* __restrict__ stop) {
  {
    const long long d = slot_delta(g);
    data = at_slot(data, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
  }
  if (stop && *stop != 0.0) return;
  constexpr int P = NYQ ? TX + 1 : TX;
  constexpr int Na = TwoPass<N>::Na, Nb = TwoPass<N>::Nb;
  constexpr int PITCH = N + 1;
  __shared__ cplx<R> A[P * PITCH];
  __shared__ cplx<R> tw[N];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const int ntiles = NYQ ? (g.n1 / 2) / TX : (g.n1h + TX - 1) / TX;
  // blocks are dispatched to the 8 XCDs in turn: when the count allows, XCD j takes a
  // contiguous range of (tile, line) units, so that the tiles of one line, whose row
  // segments share the 128-B lines at the tile boundaries, meet in that XCD's L2
  int unit = blockIdx.x;
  if ((gridDim.x & 7) == 0) unit = (unit & 7) * (gridDim.x >> 3) + (unit >> 3);
  const int tile = unit % ntiles;
  const int other = unit / ntiles;
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

hipError_t upload_reg_twiddles(hipStream_t st) {
  hipError_t e = fill_reg_twiddles(st);
  if (e == hipSuccess) e = upload_reg_twiddles_zfused(st);
  return e;
}

// ---------------------------------------------------------------------------
// Host launchers.
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
  const dim3 grid(ntiles * others, ncomp / CPB, p.nslot);
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
  const dim3 grid(ntiles * others, ncomp, p.nslot);
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
  const dim3 grid(ntiles * others, ncomp, p.nslot);
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

template <typename R, int N>
static bool launch_strided_reg(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis,
                               bool inv, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  const bool even = (g.n1 % 2 == 0);
  const int half = g.n1 / 2;
  // 16-bin tiles (more blocks in flight) measured fastest at 128^3 in both precisions
  // (FP64: 33-35 us against 34-35 at 8 bins; FP32: 18-19 us against 19-21 at 32 or 8)
  const int cap = 16;
  if (cap >= 32 && even && half % 32 == 0 && reg_lds<R>(N, 33) <= kRegLdsMax)
    launch_reg_tx<R, N, 32, true>(p, data, cs, ncomp, axis, inv, st, stop);
  else if (cap >= 16 && even && half % 16 == 0 && reg_lds<R>(N, 17) <= kRegLdsMax)
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
  const dim3 grid(ntiles * others, ncomp, p.nslot);
  hipLaunchKernelGGL((k_fft_strided<R, 0, 0>), grid, dim3(256), sm, st, data, cs, axis,
                     inv ? 1 : 0, g, pl, tw, TX, stop);
}

#define RVE_PASS_INST(R)                                                                         \
  template void launch_fft_yz<R>(const Plans&, cplx<R>*, long long, int, int, bool, hipStream_t,  \
                                 const double*);

RVE_PASS_INST(double)
RVE_PASS_INST(float)

}  // namespace rvefft
