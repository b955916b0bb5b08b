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

// Streaming access to FP64 complex fields: the non-temporal hint keeps data that a CG
// iteration touches once from displacing lines that the next kernels take from L2 and the
// Infinity Cache (the FP32 fields measured faster without it, so they load plainly).
template <typename R>
__device__ __forceinline__ cplx<R> ld_stream(const cplx<R>* p) {
  if constexpr (sizeof(R) == 8)
    return cplx<R>{__builtin_nontemporal_load(&p->x), __builtin_nontemporal_load(&p->y)};
  else
    return *p;
}
template <typename R>
__device__ __forceinline__ void st_stream(cplx<R>* p, cplx<R> v) {
  if constexpr (sizeof(R) == 8) {
    __builtin_nontemporal_store(v.x, &p->x);
    __builtin_nontemporal_store(v.y, &p->y);
  } else {
    *p = v;
  }
}

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
  int sch;                  // derivative of the momentum operator: 0 spectral (i xi~),
                            // 1 rotated finite differences (rot_factors)
  // Batched launches (several RVEs of one description in one launch): block z of the grid
  // works on RVE z, whose buffers lie sd[z] bytes from those the launch's pointer
  // arguments name (device array; nullptr: one RVE, block z = 0).
  const long long* sd = nullptr;
};

// Byte offset of this block's RVE in a batched launch, and a pointer moved by it.
__device__ __forceinline__ long long slot_delta(const Grid& g) {
  return g.sd ? g.sd[blockIdx.z] : 0;
}
template <typename T>
__device__ __forceinline__ T* at_slot(T* p, long long d) {
  return p ? reinterpret_cast<T*>(reinterpret_cast<unsigned long long>(p) + (unsigned long long)d)
           : p;
}

// Angular frequency of index k on an axis of N points and length L (signed, numpy
// ordering).  With tilde the Nyquist index of an even axis maps to zero: the
// derivative of a real field has no Nyquist component.
__device__ __forceinline__ double freq(int k, int N, double L, bool tilde) {
  if (tilde && (N % 2 == 0) && k == N / 2) return 0.0;
  const int m = (k <= (N - 1) / 2) ? k : k - N;
  return 6.283185307179586476925286766559 * (double)m / L;
}

// Rotated-scheme discrete derivative: k_a = D(theta_a) prod_{b != a} A(theta_b), the
// symbol of a forward difference along a averaged over the four parallel voxel edges,
// D = (e^{i theta} - 1) / h, A = (1 + e^{i theta}) / 2, theta = 2 pi k / N; A = 0 exactly
// at the Nyquist index (a derivative across it has no real-valued average).
__device__ __forceinline__ void rot_factors(int k, int N, double h, cplx<double>& D,
                                           cplx<double>& A) {
  double s, c;
  sincospi(2.0 * (double)k / (double)N, &s, &c);
  if (2 * k == N) { s = 0.0; c = -1.0; }
  if (k == 0) { s = 0.0; c = 1.0; }
  D = cplx<double>{(c - 1.0) / h, s / h};
  A = cplx<double>{0.5 * (1.0 + c), 0.5 * s};
}

// The three derivative symbols of bin (kx, ky, kz): i xi~ (spectral) or the rotated k.
__device__ __forceinline__ void kvec(const Grid& g, int kx, int ky, int kz, cplx<double> k[3]) {
  if (g.sch == 0) {
    k[0] = cplx<double>{0.0, freq(kx, g.n1, g.L1, true)};
    k[1] = cplx<double>{0.0, freq(ky, g.n2, g.L2, true)};
    k[2] = cplx<double>{0.0, freq(kz, g.n3, g.L3, true)};
    return;
  }
  cplx<double> Dx, Ax, Dy, Ay, Dz, Az;
  rot_factors(kx, g.n1, g.h, Dx, Ax);
  rot_factors(ky, g.n2, g.h, Dy, Ay);
  rot_factors(kz, g.n3, g.h, Dz, Az);
  k[0] = cmul(Dx, cmul(Ay, Az));
  k[1] = cmul(Ax, cmul(Dy, Az));
  k[2] = cmul(Ax, cmul(Ay, Dz));
}

__device__ __forceinline__ cplx<double> cconj(cplx<double> a) { return {a.x, -a.y}; }

// Parseval weight of a half-spectrum bin (x-bins 0 and N1/2 stand for themselves).
__device__ __forceinline__ double parseval_w(int kx, int n1) {
  return (kx == 0 || (n1 % 2 == 0 && kx == n1 / 2)) ? 1.0 : 2.0;
}

// Reduction width: one partial per block, summed in a fixed order by one block.
constexpr int kRedBlock = 256;
constexpr int kMaxRedBlocks = 2048;

}  // namespace rvefft
