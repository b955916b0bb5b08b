// Shared definitions of the HIP library: complex type, grid layout, launch checks.
//
// Layout conventions (all device fields are structure-of-arrays):
//  * a real voxel field has N = N1*N2*N3 entries, voxel (i,j,k) at i + N1*(j + N2*k);
//  * a half-spectrum field (real FFT along x) has NH = N1h*N2*N3 complex entries,
//    N1h = N1/2 + 1, bin (kx, ky, kz) at kx + N1h*(ky + N2*kz), interleaved re/im;
//  * multi-component fields store component c at offset c*N (or c*NH);
//  * symmetric tensors: components xx, yy, zz, yz, xz, xy (tensor shears); the
//    6x6 tangent is a symmetric Mandel matrix packed as its 21-entry upper triangle.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace rvefft {

template <typename R>
struct cplx {
  R x, y;
};

template <typename R>
__host__ __device__ inline cplx<R> cmul(cplx<R> a, cplx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename R>
__host__ __device__ inline cplx<R> cadd(cplx<R> a, cplx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <typename R>
__host__ __device__ inline cplx<R> csub(cplx<R> a, cplx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <typename R>
__host__ __device__ inline cplx<R> cscale(cplx<R> a, R s) { return {a.x * s, a.y * s}; }

// Up to 6 radix-2/3/4 stages cover every length 2^a 3^b <= 4096.
constexpr int kMaxStages = 8;
constexpr int kMaxN = 512;

struct AxisPlan {
  int n;                    // transform length
  int nst;                  // number of stages
  int radix[kMaxStages];    // radices in stage order
};

struct Grid {
  int n1, n2, n3;
  int n1h;                  // n1/2 + 1
  long long nvox;           // n1*n2*n3
  long long nspec;          // n1h*n2*n3
  double h;                 // voxel edge [m]
  double L1, L2, L3;        // box lengths [m]
};

// Angular frequency of index k on an axis of N points and length L (signed, numpy
// ordering).  With tilde the Nyquist index of an even axis maps to zero: the
// derivative of a real field has no Nyquist component.
__device__ __forceinline__ double freq(int k, int N, double L, bool tilde) {
  if (tilde && (N % 2 == 0) && k == N / 2) return 0.0;
  const int m = (k <= (N - 1) / 2) ? k : k - N;
  return 6.283185307179586476925286766559 * (double)m / L;
}

// Parseval weight of a half-spectrum bin (x-bins 0 and N1/2 stand for themselves).
__device__ __forceinline__ double parseval_w(int kx, int n1) {
  return (kx == 0 || (n1 % 2 == 0 && kx == n1 / 2)) ? 1.0 : 2.0;
}

// Reduction width: one partial per block, summed in a fixed order by one block.
constexpr int kRedBlock = 256;
constexpr int kMaxRedBlocks = 2048;

}  // namespace rvefft
