// Phase-field balance (eqs. strpf and phase) with the pre-set crack held at phi = 1 as a
// Dirichlet condition: phi = u + 1_crack, u = 0 on the crack and P A P u = P (2S - A 1_crack)
// on the free voxels, A = (1 + 2S) - l^2 lap.  The crack is the set of voxels that cannot
// slip (infinite slip resistance): the geometric crack or soft buffer of Secs. 4.1 and 4.5,
// given as phi0 = 1.  Pointwise kernels of the conjugate-gradient loop; the Laplacian and
// the preconditioner are FFT round trips.
#include "kernels.h"

namespace rvefft {

namespace {
int pgrid(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}
}  // namespace

__global__ void __launch_bounds__(256) k_pfd(long long N, int mode, const double* __restrict__ x,
                                             const double* __restrict__ w,
                                             const double* __restrict__ S,
                                             const double* __restrict__ gslip,
                                             double* __restrict__ y,
                                             const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const bool fr = isfinite(gslip[v]);
    double r;
    switch (mode) {
      case 0: r = fr ? x[v] : 0.0; break;
      case 1: r = fr ? 0.0 : 1.0; break;
      case 2: r = fr ? (1.0 + 2.0 * S[v]) * x[v] + w[v] : 0.0; break;
      default: r = fr ? 2.0 * S[v] - ((1.0 + 2.0 * S[v]) * x[v] + w[v]) : 0.0; break;
    }
    y[v] = r;
  }
}

__global__ void __launch_bounds__(256) k_pfd_axpy(long long N, const double* __restrict__ sc,
                                                  int ia, int ib, double sign,
                                                  const double* __restrict__ x,
                                                  double* __restrict__ y,
                                                  const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  const double a = sc ? sign * sc[ia] / sc[ib] : sign;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
    y[v] += a * x[v];
}

__global__ void __launch_bounds__(256) k_pfd_xpby(long long N, const double* __restrict__ z,
                                                  const double* __restrict__ sc, int ia, int ib,
                                                  double* __restrict__ p,
                                                  const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  const double b = sc[ia] / sc[ib];
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
    p[v] = z[v] + b * p[v];
}

void launch_pfd(long long N, int mode, const double* x, const double* w, const double* S,
                const double* gslip, double* y, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL(k_pfd, dim3(pgrid(N)), dim3(256), 0, st, N, mode, x, w, S, gslip, y, stop);
}
void launch_pfd_axpy(long long N, const double* sc, int ia, int ib, double sign, const double* x,
                     double* y, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL(k_pfd_axpy, dim3(pgrid(N)), dim3(256), 0, st, N, sc, ia, ib, sign, x, y,
                     stop);
}
void launch_pfd_xpby(long long N, const double* z, const double* sc, int ia, int ib, double* p,
                     hipStream_t st, const double* stop) {
  hipLaunchKernelGGL(k_pfd_xpby, dim3(pgrid(N)), dim3(256), 0, st, N, z, sc, ia, ib, p, stop);
}

}  // namespace rvefft
