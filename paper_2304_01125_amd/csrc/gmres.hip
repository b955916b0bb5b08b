// Vector kernels of the restarted GMRES(m) option of the momentum Krylov solve (the
// paper's solver, Sec. 3.1 with eq. newton): several Parseval-weighted dot products of
// one vector with a block of basis vectors in one pass, the matching block update, and
// scalings.  Vectors are 3-component half spectra; the inner product is the real one of
// the half spectrum weighted 1 on the x-bins 0 and N1/2 and 2 elsewhere.
#include "kernels.h"

namespace rvefft {

namespace {

__device__ __forceinline__ double gm_weight(long long b, const Grid& g) {
  const int kx = (int)((unsigned)b % (unsigned)g.n1h);
  return (kx == 0 || (g.n1 % 2 == 0 && kx == g.n1 / 2)) ? 1.0 : 2.0;
}

int gm_grid(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < kMaxRedBlocks ? (b < 1 ? 1 : b) : kMaxRedBlocks);
}

}  // namespace

// partial[i * gridDim + blk] = block sums of <V_i, w>, i < nv <= kGmChunk
template <typename R>
__global__ void __launch_bounds__(256)
k_mdot(const cplx<R>* __restrict__ V, long long vs, int nv, const cplx<R>* __restrict__ w,
       long long cs, Grid g, double* __restrict__ partial) {
  __shared__ double red[kGmChunk][4];
  double acc[kGmChunk];
#pragma unroll
  for (int i = 0; i < kGmChunk; ++i) acc[i] = 0.0;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const double pw = gm_weight(b, g);
    const cplx<R> w0 = w[b], w1 = w[cs + b], w2 = w[2 * cs + b];
#pragma unroll
    for (int i = 0; i < kGmChunk; ++i) {
      if (i < nv) {
        const cplx<R>* v = V + i * vs;
        const cplx<R> a = v[b], c = v[cs + b], d = v[2 * cs + b];
        const double s = (double)a.x * w0.x + (double)a.y * w0.y + (double)c.x * w1.x +
                         (double)c.y * w1.y + (double)d.x * w2.x + (double)d.y * w2.y;
        acc[i] += pw * s;
      }
    }
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < kGmChunk; ++i) {
    double x = acc[i];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) red[i][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < nv) {
    const int i = threadIdx.x;
    partial[(long long)i * gridDim.x + blockIdx.x] = red[i][0] + red[i][1] + red[i][2] + red[i][3];
  }
}

// w += sum_i coef[i] V_i, i < nv <= kGmChunk (coef: device doubles)
template <typename R>
__global__ void __launch_bounds__(256)
k_maxpy(const cplx<R>* __restrict__ V, long long vs, int nv, const double* __restrict__ coef,
        double sign, cplx<R>* __restrict__ w, long long cs, long long n) {
  double a[kGmChunk];
#pragma unroll
  for (int i = 0; i < kGmChunk; ++i) a[i] = (i < nv) ? sign * coef[i] : 0.0;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < n;
       b += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long j = c * cs + b;
      double x = (double)w[j].x, y = (double)w[j].y;
#pragma unroll
      for (int i = 0; i < kGmChunk; ++i)
        if (i < nv) {
          const cplx<R> v = V[i * vs + j];
          x += a[i] * (double)v.x;
          y += a[i] * (double)v.y;
        }
      w[j] = cplx<R>{(R)x, (R)y};
    }
  }
}

// out = a * in + b * y (3 components; y may be null when b = 0)
template <typename R>
__global__ void __launch_bounds__(256)
k_caxpby(const cplx<R>* __restrict__ in, double a, const cplx<R>* __restrict__ y, double bco,
         cplx<R>* __restrict__ out, long long cs, long long n) {
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < n;
       b += (long long)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long j = c * cs + b;
      double x = a * (double)in[j].x, z = a * (double)in[j].y;
      if (y) {
        x += bco * (double)y[j].x;
        z += bco * (double)y[j].y;
      }
      out[j] = cplx<R>{(R)x, (R)z};
    }
}

template <typename R>
int launch_mdot(const Plans& p, const cplx<R>* V, long long vs, int nv, const cplx<R>* w,
                long long cs, double* partial, hipStream_t st) {
  const int nb = gm_grid(p.g.nspec);
  hipLaunchKernelGGL((k_mdot<R>), dim3(nb), dim3(256), 0, st, V, vs, nv, w, cs, p.g, partial);
  return nb;
}
template <typename R>
void launch_maxpy(const Plans& p, const cplx<R>* V, long long vs, int nv, const double* coef,
                  double sign, cplx<R>* w, long long cs, hipStream_t st) {
  hipLaunchKernelGGL((k_maxpy<R>), dim3(gm_grid(p.g.nspec)), dim3(256), 0, st, V, vs, nv, coef,
                     sign, w, cs, p.g.nspec);
}
template <typename R>
void launch_caxpby(const Plans& p, const cplx<R>* in, double a, const cplx<R>* y, double b,
                   cplx<R>* out, long long cs, hipStream_t st) {
  hipLaunchKernelGGL((k_caxpby<R>), dim3(gm_grid(p.g.nspec)), dim3(256), 0, st, in, a, y, b, out,
                     cs, p.g.nspec);
}

#define RVE_GMRES_INST(R)                                                                        \
  template int launch_mdot<R>(const Plans&, const cplx<R>*, long long, int, const cplx<R>*,       \
                              long long, double*, hipStream_t);                                  \
  template void launch_maxpy<R>(const Plans&, const cplx<R>*, long long, int, const double*,      \
                                double, cplx<R>*, long long, hipStream_t);                       \
  template void launch_caxpby<R>(const Plans&, const cplx<R>*, double, const cplx<R>*, double,    \
                                 cplx<R>*, long long, hipStream_t);

RVE_GMRES_INST(double)
RVE_GMRES_INST(float)

}  // namespace rvefft
