// Mixed-radix (2, 3, 4) Stockham FFT of pencils held in LDS.
//
// The discrete Fourier transforms of Sec. 3.1 (fields at voxel centres, FFT of
// every component) are computed by batches of 1-D transforms along x (real rows,
// two rows packed into one complex pencil), then y and z (strided complex
// pencils).  Forward transforms use exp(-2 pi i k n / N), inverse ones
// exp(+2 pi i k n / N); neither is normalised.
#pragma once
#include "common.h"

namespace rvefft {

// In-register DFT of size r (2, 3 or 4) of v[0..r-1].
template <typename R>
__device__ __forceinline__ void small_dft(cplx<R>* v, int r, bool inv) {
  if (r == 2) {
    cplx<R> a = v[0], b = v[1];
    v[0] = cadd(a, b);
    v[1] = csub(a, b);
  } else if (r == 4) {
    cplx<R> a = v[0], b = v[1], c = v[2], d = v[3];
    cplx<R> s0 = cadd(a, c), s1 = csub(a, c), s2 = cadd(b, d), s3 = csub(b, d);
    // forward: y1 = s1 - i s3, y3 = s1 + i s3 ; inverse swaps the sign of i
    cplx<R> is3 = {-s3.y, s3.x};               // i * s3
    v[0] = cadd(s0, s2);
    v[2] = csub(s0, s2);
    if (!inv) {
      v[1] = csub(s1, is3);
      v[3] = cadd(s1, is3);
    } else {
      v[1] = cadd(s1, is3);
      v[3] = csub(s1, is3);
    }
  } else if (r == 3) {
    const R h = R(0.86602540378443864676);    // sqrt(3)/2
    cplx<R> a = v[0], b = v[1], c = v[2];
    cplx<R> t1 = cadd(b, c);
    cplx<R> t2 = {a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y};
    cplx<R> d = csub(b, c);
    // forward: y1 = t2 - i h d, y2 = t2 + i h d
    cplx<R> ihd = {-h * d.y, h * d.x};
    v[0] = cadd(a, t1);
    if (!inv) {
      v[1] = csub(t2, ihd);
      v[2] = cadd(t2, ihd);
    } else {
      v[1] = cadd(t2, ihd);
      v[2] = csub(t2, ihd);
    }
  }
}

// Transform P pencils of length pl.n stored in LDS buffer `a` (element (n, p) at
// n*sn + p*sp), using `b` (same layout) as the Stockham ping-pong partner.  `tw`
// holds exp(-2 pi i k / n), k < n.  Returns the buffer that holds the result.
// All threads of the block must call it; it ends with a barrier.
// PFAST selects the thread mapping: consecutive threads on consecutive pencils
// (true, for pencil-fastest layouts) or on consecutive butterflies (false).
template <typename R, bool PFAST>
__device__ cplx<R>* fft_pencils(cplx<R>* a, cplx<R>* b, const cplx<R>* tw, const AxisPlan& pl,
                                int P, int sn, int sp, bool inv) {
  const int N = pl.n;
  int Ns = 1;
  for (int s = 0; s < pl.nst; ++s) {
    const int r = pl.radix[s];
    const int nb = N / r;
    const int tstride = N / (Ns * r);
    for (int t = threadIdx.x; t < nb * P; t += blockDim.x) {
      int p, j;
      if (PFAST) { p = t % P; j = t / P; } else { j = t % nb; p = t / nb; }
      const int k = j % Ns;
      cplx<R> v[4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < r) v[q] = a[(j + q * nb) * sn + p * sp];
#pragma unroll
      for (int q = 1; q < 4; ++q) {
        if (q < r) {
          cplx<R> w = tw[q * k * tstride];
          if (inv) w.y = -w.y;
          v[q] = cmul(v[q], w);
        }
      }
      small_dft(v, r, inv);
      const int idxD = (j / Ns) * Ns * r + k;
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if (q < r) b[(idxD + q * Ns) * sn + p * sp] = v[q];
    }
    __syncthreads();
    cplx<R>* t = a; a = b; b = t;
    Ns *= r;
  }
  return a;
}

// ---- compile-time lengths ---------------------------------------------------------
// Radix of stage s of the schedule used for length n (4s first, then 2, then 3s) and
// the number of stages; identical to make_axis_plan.
constexpr int ct_radix(int n, int s) {
  int m = n, k = 0;
  while (m % 4 == 0) { if (k == s) return 4; m /= 4; ++k; }
  while (m % 2 == 0) { if (k == s) return 2; m /= 2; ++k; }
  while (m % 3 == 0) { if (k == s) return 3; m /= 3; ++k; }
  return 1;
}
constexpr int ct_nstages(int n) {
  int m = n, k = 0;
  while (m % 4 == 0) { m /= 4; ++k; }
  while (m % 2 == 0) { m /= 2; ++k; }
  while (m % 3 == 0) { m /= 3; ++k; }
  return k;
}

// One Stockham stage with every size known at compile time.  Layout: element (n, p)
// at n*SN + p*SP.  P pencils; PFAST as in fft_pencils.  P may be 0 for "runtime P"
// (only with PFAST = false, where no division by P is needed).
template <typename R, int N, int S, int NS, int SN, int SP, int PCT, bool PFAST>
__device__ __forceinline__ void ct_stage(const cplx<R>* __restrict__ a, cplx<R>* __restrict__ b,
                                         const cplx<R>* __restrict__ tw, int P, bool inv) {
  constexpr int r = ct_radix(N, S);
  constexpr int nb = N / r;
  constexpr int tstride = N / (NS * r);
  const int Pn = PCT ? PCT : P;
  const int sp = SP ? SP : 0;
  for (int t = threadIdx.x; t < nb * Pn; t += blockDim.x) {
    int p, j;
    if constexpr (PFAST) { p = t % PCT; j = t / PCT; } else { j = t % nb; p = t / nb; }
    const int k = j % NS;
    cplx<R> v[4];
#pragma unroll
    for (int q = 0; q < r; ++q) v[q] = a[(j + q * nb) * SN + p * sp];
#pragma unroll
    for (int q = 1; q < r; ++q) {
      cplx<R> w = tw[q * k * tstride];
      if (inv) w.y = -w.y;
      v[q] = cmul(v[q], w);
    }
    small_dft(v, r, inv);
    const int idxD = (j / NS) * NS * r + k;
#pragma unroll
    for (int q = 0; q < r; ++q) b[(idxD + q * NS) * SN + p * sp] = v[q];
  }
}

template <typename R, int N, int S, int NS, int SN, int SP, int PCT, bool PFAST>
__device__ __forceinline__ cplx<R>* ct_run(cplx<R>* a, cplx<R>* b, const cplx<R>* tw, int P,
                                           bool inv) {
  if constexpr (S == ct_nstages(N)) {
    return a;
  } else {
    ct_stage<R, N, S, NS, SN, SP, PCT, PFAST>(a, b, tw, P, inv);
    __syncthreads();
    return ct_run<R, N, S + 1, NS * ct_radix(N, S), SN, SP, PCT, PFAST>(b, a, tw, P, inv);
  }
}

// TX pencils of length N in layout [n][TX] (pencil fastest): strided passes.
template <typename R, int N, int TX>
__device__ __forceinline__ cplx<R>* fft_tiles_ct(cplx<R>* a, cplx<R>* b, const cplx<R>* tw,
                                                 bool inv) {
  return ct_run<R, N, 0, 1, TX, 1, TX, true>(a, b, tw, TX, inv);
}

// P pencils of length N in layout [p][N+1] (row fastest): x passes.
template <typename R, int N>
__device__ __forceinline__ cplx<R>* fft_rows_ct(cplx<R>* a, cplx<R>* b, const cplx<R>* tw, int P,
                                                bool inv) {
  return ct_run<R, N, 0, 1, 1, N + 1, 0, false>(a, b, tw, P, inv);
}

// ---- in-place (single LDS buffer) stages ------------------------------------------
// Each thread first reads the inputs of all its butterflies into registers, the block
// synchronises, then every thread writes its outputs over the same buffer: half the
// LDS of a ping-pong pair, hence twice the resident blocks.  NT = block size.
template <typename R, int N, int S, int NS, int SN, int SP, int P, bool PFAST, int NT>
__device__ __forceinline__ void ct_stage_ip(cplx<R>* __restrict__ a, const cplx<R>* __restrict__ tw,
                                            bool inv) {
  constexpr int r = ct_radix(N, S);
  constexpr int nb = N / r;
  constexpr int tstride = N / (NS * r);
  constexpr int total = nb * P;
  constexpr int per = (total + NT - 1) / NT;
  cplx<R> v[per][4];
#pragma unroll
  for (int u = 0; u < per; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t < total) {
      int p, j;
      if constexpr (PFAST) { p = t % P; j = t / P; } else { j = t % nb; p = t / nb; }
#pragma unroll
      for (int q = 0; q < r; ++q) v[u][q] = a[(j + q * nb) * SN + p * SP];
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < per; ++u) {
    const int t = threadIdx.x + u * NT;
    if (t < total) {
      int p, j;
      if constexpr (PFAST) { p = t % P; j = t / P; } else { j = t % nb; p = t / nb; }
      const int k = j % NS;
#pragma unroll
      for (int q = 1; q < r; ++q) {
        cplx<R> w = tw[q * k * tstride];
        if (inv) w.y = -w.y;
        v[u][q] = cmul(v[u][q], w);
      }
      small_dft(v[u], r, inv);
      const int idxD = (j / NS) * NS * r + k;
#pragma unroll
      for (int q = 0; q < r; ++q) a[(idxD + q * NS) * SN + p * SP] = v[u][q];
    }
  }
  __syncthreads();
}

template <typename R, int N, int S, int NS, int SN, int SP, int P, bool PFAST, int NT>
__device__ __forceinline__ void ct_run_ip(cplx<R>* a, const cplx<R>* tw, bool inv) {
  if constexpr (S < ct_nstages(N)) {
    ct_stage_ip<R, N, S, NS, SN, SP, P, PFAST, NT>(a, tw, inv);
    ct_run_ip<R, N, S + 1, NS * ct_radix(N, S), SN, SP, P, PFAST, NT>(a, tw, inv);
  }
}

// In-place transforms: TX pencils in [n][TX] layout, or P rows in [p][N+1] layout.
template <typename R, int N, int TX, int NT>
__device__ __forceinline__ void fft_tiles_ip(cplx<R>* a, const cplx<R>* tw, bool inv) {
  ct_run_ip<R, N, 0, 1, TX, 1, TX, true, NT>(a, tw, inv);
}
template <typename R, int N, int P, int NT>
__device__ __forceinline__ void fft_rows_ip(cplx<R>* a, const cplx<R>* tw, bool inv) {
  ct_run_ip<R, N, 0, 1, 1, N + 1, P, false, NT>(a, tw, inv);
}

}  // namespace rvefft
