// Register-resident DFTs and the two-pass (Na x Nb) pencil FFT.
//
// A length-N transform (N = Na * Nb) of a pencil x[n] is done in two passes:
//   pass 1: for each n1 < Nb, the Na values x[n1 + Nb m] are transformed in registers,
//           multiplied by exp(-+2 pi i n1 k2 / N) and stored to LDS at n1 + Nb k2;
//   pass 2: for each k2 < Na, the Nb values at n1 + Nb k2 are transformed in registers
//           and give X[k2 + Na k1], k1 < Nb.
// Every small DFT is fully unrolled; its twiddles are compile-time table entries.
#pragma once
#include "common.h"
#include <cmath>

namespace rvefft {

// exp(-2 pi i k / 256) and exp(-2 pi i k / 192), k < 256 / 192: every register DFT
// length used here divides one of them.  The library is built without relocatable
// device code, so each translation unit that uses the register DFTs holds its own copy
// of the tables and fills it with its own fill_reg_twiddles (at handle creation).
static __constant__ double c_tw256[2 * 256];
static __constant__ double c_tw192[2 * 192];

static inline hipError_t fill_reg_twiddles(hipStream_t st) {
  double t256[512], t192[384];
  for (int k = 0; k < 256; ++k) {
    t256[2 * k] = std::cos(-2.0 * M_PI * k / 256.0);
    t256[2 * k + 1] = std::sin(-2.0 * M_PI * k / 256.0);
  }
  for (int k = 0; k < 192; ++k) {
    t192[2 * k] = std::cos(-2.0 * M_PI * k / 192.0);
    t192[2 * k + 1] = std::sin(-2.0 * M_PI * k / 192.0);
  }
  hipError_t e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tw256), t256, sizeof(t256), 0,
                                        hipMemcpyHostToDevice, st);
  if (e == hipSuccess)
    e = hipMemcpyToSymbolAsync(HIP_SYMBOL(c_tw192), t192, sizeof(t192), 0, hipMemcpyHostToDevice,
                               st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  return e;
}

template <typename R, int L>
__device__ __forceinline__ cplx<R> ctw(int a) {   // exp(-2 pi i a / L), a compile-time
  if constexpr (256 % L == 0) {
    const int k = (a % L) * (256 / L);
    return cplx<R>{(R)c_tw256[2 * k], (R)c_tw256[2 * k + 1]};
  } else {
    static_assert(192 % L == 0, "register DFT length must divide 256 or 192");
    const int k = (a % L) * (192 / L);
    return cplx<R>{(R)c_tw192[2 * k], (R)c_tw192[2 * k + 1]};
  }
}

template <typename R, bool INV>
__device__ __forceinline__ void rdft2(cplx<R>* v) {
  const cplx<R> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <typename R, bool INV>
__device__ __forceinline__ void rdft3(cplx<R>* v) {
  const R h = R(0.86602540378443864676);
  const cplx<R> a = v[0], b = v[1], c = v[2];
  const cplx<R> t1 = cadd(b, c);
  const cplx<R> t2 = {a.x - R(0.5) * t1.x, a.y - R(0.5) * t1.y};
  const cplx<R> d = csub(b, c);
  const cplx<R> ihd = {-h * d.y, h * d.x};
  v[0] = cadd(a, t1);
  if constexpr (!INV) { v[1] = csub(t2, ihd); v[2] = cadd(t2, ihd); }
  else { v[1] = cadd(t2, ihd); v[2] = csub(t2, ihd); }
}
template <typename R, bool INV>
__device__ __forceinline__ void rdft4(cplx<R>* v) {
  const cplx<R> s0 = cadd(v[0], v[2]), s1 = csub(v[0], v[2]), s2 = cadd(v[1], v[3]),
                s3 = csub(v[1], v[3]);
  const cplx<R> is3 = {-s3.y, s3.x};
  v[0] = cadd(s0, s2);
  v[2] = csub(s0, s2);
  if constexpr (!INV) { v[1] = csub(s1, is3); v[3] = cadd(s1, is3); }
  else { v[1] = cadd(s1, is3); v[3] = csub(s1, is3); }
}

// In-register DFT of length L (products of 2, 3, 4), decimation in time:
// X[k2 + m k1] = sum_n1 W_r^{n1 k1} W_L^{n1 k2} DFT_m(x[r n2 + n1])[k2],  L = r m.
template <typename R, int L, bool INV>
__device__ __forceinline__ void reg_dft(cplx<R>* v) {
  if constexpr (L == 1) {
  } else if constexpr (L == 2) {
    rdft2<R, INV>(v);
  } else if constexpr (L == 3) {
    rdft3<R, INV>(v);
  } else if constexpr (L == 4) {
    rdft4<R, INV>(v);
  } else {
    constexpr int r = (L % 4 == 0) ? 4 : ((L % 2 == 0) ? 2 : 3);
    constexpr int m = L / r;
    cplx<R> sub[r][m];
#pragma unroll
    for (int n1 = 0; n1 < r; ++n1)
#pragma unroll
      for (int n2 = 0; n2 < m; ++n2) sub[n1][n2] = v[r * n2 + n1];
#pragma unroll
    for (int n1 = 0; n1 < r; ++n1) reg_dft<R, m, INV>(sub[n1]);
#pragma unroll
    for (int k2 = 0; k2 < m; ++k2) {
      cplx<R> t[r];
#pragma unroll
      for (int n1 = 0; n1 < r; ++n1) {
        if (n1 * k2 == 0) {
          t[n1] = sub[n1][k2];
        } else {
          cplx<R> w = ctw<R, L>(n1 * k2);
          if constexpr (INV) w.y = -w.y;
          t[n1] = cmul(sub[n1][k2], w);
        }
      }
      if constexpr (r == 2) rdft2<R, INV>(t);
      else if constexpr (r == 3) rdft3<R, INV>(t);
      else rdft4<R, INV>(t);
#pragma unroll
      for (int k1 = 0; k1 < r; ++k1) v[k2 + m * k1] = t[k1];
    }
  }
}

// Split of each supported length into Na x Nb for the two-pass FFT.
template <int N> struct TwoPass;
template <> struct TwoPass<16> { static constexpr int Na = 4, Nb = 4; };
template <> struct TwoPass<32> { static constexpr int Na = 8, Nb = 4; };
template <> struct TwoPass<48> { static constexpr int Na = 16, Nb = 3; };
template <> struct TwoPass<64> { static constexpr int Na = 8, Nb = 8; };
template <> struct TwoPass<96> { static constexpr int Na = 16, Nb = 6; };
template <> struct TwoPass<128> { static constexpr int Na = 16, Nb = 8; };
template <> struct TwoPass<256> { static constexpr int Na = 16, Nb = 16; };

}  // namespace rvefft
