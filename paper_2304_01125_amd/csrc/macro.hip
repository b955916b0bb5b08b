// Mixed strain/stress macroscopic control (the DBFFT mixed extension the method relies
// on, Sec. 3.1).  The macro strain components under stress control are unknowns of the
// momentum Newton-Krylov system.  They ride in the zero-frequency bin of the
// 3-component half-spectrum vectors, whose six reals hold the Mandel values
//   x: (xx, xy), y: (yy, yz), z: (zz, xz).
// The operator maps them to the zero-frequency strain s E (real-space macro strain
// s E / N) and returns q(0) = s sigma^_M(0) on the stress-controlled components, with
// s = N xi_1 (xi_1 = 2 pi / L_max, the lowest frequency, so that the macro rows carry the
// units of the fluctuation rows).  In the Parseval inner product the extended operator is
// the Hessian of sum_v g w(eps) - N sigma* . E_F: symmetric positive definite, and CG
// applies unchanged; its preconditioner on the macro block is (s^2 Kbar_FF)^-1.
#include "kernels.h"

namespace rvefft {

namespace {

constexpr double kS2 = 1.41421356237309504880, kIS2 = 0.70710678118654752440;

// Mandel index -> vector component and real (0) / imaginary (1) part of the zero bin
__device__ __forceinline__ int mslot_comp(int c) { return c < 3 ? c : (c == 3 ? 1 : (c == 4 ? 2 : 0)); }
__device__ __forceinline__ int mslot_im(int c) { return c < 3 ? 0 : 1; }

template <typename R>
__device__ __forceinline__ double mget(const cplx<R>* v, long long cs, int c) {
  const cplx<R> a = v[mslot_comp(c) * cs];
  return mslot_im(c) ? (double)a.y : (double)a.x;
}

template <typename R>
__device__ __forceinline__ void mput(cplx<R>* v, long long cs, const double m[6]) {
  v[0] = cplx<R>{(R)m[0], (R)m[5]};
  v[cs] = cplx<R>{(R)m[1], (R)m[3]};
  v[2 * cs] = cplx<R>{(R)m[2], (R)m[4]};
}

__device__ __forceinline__ constexpr int pk6(int i, int j) {
  return (i <= j) ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j);
}

}  // namespace

// e_c += s E_c (tensor component: Mandel value / sqrt 2 for shears) on the stress-
// controlled components: at the zero-frequency bin (nz = 1), or along the (0, 0) z column
// when the z axis is still spatial (an inverse z transform turns a zero-frequency value
// into that value at every z).  de_out (optional): the real-space macro strain
// increment (s / N) E (Mandel), 0 on the strain-controlled components.
template <typename R>
__global__ void __launch_bounds__(256)
k_macro_strain(cplx<R>* __restrict__ e, long long ecs, const cplx<R>* __restrict__ pv,
               long long pcs, double s, double de_scale, int mask, int nz, long long zstride,
               double* __restrict__ de_out, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (int t = threadIdx.x; t < 6 * nz; t += blockDim.x) {
    const int c = t % 6, z = t / 6;
    if (!((mask >> c) & 1)) continue;
    const double v = s * mget(pv, pcs, c) * (c < 3 ? 1.0 : kIS2);
    cplx<R>& a = e[c * ecs + (long long)z * zstride];
    a.x = (R)((double)a.x + v);
  }
  if (de_out && threadIdx.x < 6) {
    const int c = threadIdx.x;
    de_out[c] = ((mask >> c) & 1) ? de_scale * mget(pv, pcs, c) : 0.0;
  }
}

// q(0) = s sigma^_M(0) on the stress-controlled components (0 on the others) and the
// zero-frequency term of <p, q> at pq_out.  sigma^(0) is the sum of the (0, 0) z column
// when z is still spatial (nz = N3), else the zero-frequency bin (nz = 1).
// One wave per component: lanes take every 64th z, then a fixed-order shuffle sum.
template <typename R>
__global__ void __launch_bounds__(384)
k_macro_stress(const cplx<R>* __restrict__ sg, long long scs, cplx<R>* __restrict__ q,
               const cplx<R>* __restrict__ pv, long long cs, double s, int mask, int nz,
               long long zstride, double* __restrict__ pq_out, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double qm[6];
  const int c = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double sum = 0.0;
  for (int z = lane; z < nz; z += 64) sum += (double)sg[c * scs + (long long)z * zstride].x;
  for (int off = 32; off > 0; off >>= 1) sum += __shfl_down(sum, off, 64);
  if (lane == 0) qm[c] = ((mask >> c) & 1) ? s * sum * (c < 3 ? 1.0 : kS2) : 0.0;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m[6], pq = 0.0;
    for (int c = 0; c < 6; ++c) {
      m[c] = qm[c];
      pq += mget(pv, cs, c) * qm[c];
    }
    mput(q, cs, m);
    *pq_out = pq;
  }
}

// Right-hand side at the zero bin: b(0) = -s (sigma^_M(0) - N sigma*_M) on the stress-
// controlled components, from the full spectrum of g sigma.
template <typename R>
__global__ void __launch_bounds__(64)
k_macro_rhs(const cplx<R>* __restrict__ sg, long long scs, cplx<R>* __restrict__ b, long long cs,
            double s, double n, Six6 tgt, int mask) {
  if (threadIdx.x != 0) return;
  double m[6];
  for (int c = 0; c < 6; ++c) {
    const double sm = (double)sg[c * scs].x * (c < 3 ? 1.0 : kS2);
    m[c] = ((mask >> c) & 1) ? -s * (sm - n * tgt.v[c]) : 0.0;
  }
  mput(b, cs, m);
}

// M0 = (s^2 Kbar_FF)^-1 on the stress-controlled components (6 x 6, zero elsewhere): the
// strain-controlled rows and columns are replaced by those of the identity, the 6 x 6 is
// inverted by Gauss-Jordan elimination without pivoting (symmetric positive definite),
// fully unrolled so that it stays in registers, and those rows and columns are cleared.
// The block s^2 Kbar_FF itself follows (the CG step recovers r(0) = M0^-1 z(0) with it).
__global__ void __launch_bounds__(64)
k_macro_prec(const double* __restrict__ kbar21, double s2, int mask, double* __restrict__ m0) {
  if (threadIdx.x != 0) return;
  double A[6][6], B[6][6];
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const bool fi = (mask >> i) & 1, fj = (mask >> j) & 1;
      A[i][j] = (fi && fj) ? s2 * kbar21[pk6(i, j)] : (i == j ? 1.0 : 0.0);
      B[i][j] = (i == j) ? 1.0 : 0.0;
    }
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const double d = 1.0 / A[k][k];
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      A[k][j] *= d;
      B[k][j] *= d;
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      if (i == k) continue;
      const double f = A[i][k];
#pragma unroll
      for (int j = 0; j < 6; ++j) {
        A[i][j] -= f * A[k][j];
        B[i][j] -= f * B[k][j];
      }
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = 0; j < 6; ++j) {
      const bool f = ((mask >> i) & 1) && ((mask >> j) & 1);
      m0[i * 6 + j] = f ? B[i][j] : 0.0;
      m0[36 + i * 6 + j] = f ? s2 * kbar21[pk6(i, j)] : 0.0;   // the block itself
    }
}

template <typename R>
void launch_macro_strain(cplx<R>* e, long long ecs, const cplx<R>* pv, long long pcs, double s,
                         double de_scale, int mask, int nz, long long zstride, double* de_out,
                         hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_macro_strain<R>), dim3(1), dim3(256), 0, st, e, ecs, pv, pcs, s, de_scale,
                     mask, nz, zstride, de_out, stop);
}
template <typename R>
void launch_macro_stress(const cplx<R>* sg, long long scs, cplx<R>* q, const cplx<R>* pv,
                         long long cs, double s, int mask, int nz, long long zstride,
                         double* pq_out, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_macro_stress<R>), dim3(1), dim3(384), 0, st, sg, scs, q, pv, cs, s, mask,
                     nz, zstride, pq_out, stop);
}
template <typename R>
void launch_macro_rhs(const cplx<R>* sg, long long scs, cplx<R>* b, long long cs, double s,
                      double n, const double tgt[6], int mask, hipStream_t st) {
  Six6 t;
  for (int c = 0; c < 6; ++c) t.v[c] = tgt[c];
  hipLaunchKernelGGL((k_macro_rhs<R>), dim3(1), dim3(64), 0, st, sg, scs, b, cs, s, n, t, mask);
}
void launch_macro_prec(const double* kbar21, double s2, int mask, double* m0, hipStream_t st) {
  hipLaunchKernelGGL(k_macro_prec, dim3(1), dim3(64), 0, st, kbar21, s2, mask, m0);
}

#define RVE_MACRO_INST(R)                                                                        \
  template void launch_macro_strain<R>(cplx<R>*, long long, const cplx<R>*, long long, double,    \
                                       double, int, int, long long, double*, hipStream_t,         \
                                       const double*);                                           \
  template void launch_macro_stress<R>(const cplx<R>*, long long, cplx<R>*, const cplx<R>*,       \
                                       long long, double, int, int, long long, double*,           \
                                       hipStream_t, const double*);                              \
  template void launch_macro_rhs<R>(const cplx<R>*, long long, cplx<R>*, long long, double,       \
                                    double, const double*, int, hipStream_t);

RVE_MACRO_INST(double)
RVE_MACRO_INST(float)

}  // namespace rvefft
