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

}  // namespace rvefft
