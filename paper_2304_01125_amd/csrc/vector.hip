// Krylov vector kernels and deterministic reductions.
//
// The momentum Krylov space is the real vector space of half-spectrum displacement
// corrections; its inner product weights every bin by its multiplicity in the full
// spectrum (1 on the x-bins 0 and N1/2, 2 elsewhere), i.e. Parseval's identity for
// the real fields they represent.  All dot products accumulate in FP64; every
// reduction is a fixed tree (per-block partials, then one block in index order), so
// results are bitwise reproducible run to run.
#include "kernels.h"

namespace rvefft {

static int vgrid(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

__global__ void __launch_bounds__(256) k_reduce(const double* __restrict__ partial, int nblk, int op_max,
                         double* __restrict__ out, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double sh[256];
  const int c = blockIdx.x;
  double s = op_max ? -INFINITY : 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const double x = partial[(long long)c * nblk + b];
    s = op_max ? fmax(s, x) : s + x;
  }
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = blockDim.x / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) {
      const double y = sh[threadIdx.x + w];
      sh[threadIdx.x] = op_max ? fmax(sh[threadIdx.x], y) : sh[threadIdx.x] + y;
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = sh[0];
}

void launch_reduce(const double* partial, int nblk, int ncomp, int op_max, double* out,
                   hipStream_t st, const double* stop) {
  hipLaunchKernelGGL(k_reduce, dim3(ncomp), dim3(256), 0, st, partial, nblk, op_max, out, stop);
}

// Fixed-order sum of a[0..n) by one block of 256 threads (result valid in thread 0).
__device__ double block_sum256(const double* __restrict__ a, int n, double* sh) {
  double s = 0.0;
  for (int b = threadIdx.x; b < n; b += 256) s += a[b];
  sh[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w) sh[threadIdx.x] += sh[threadIdx.x + w];
    __syncthreads();
  }
  return sh[0];
}

__global__ void __launch_bounds__(256) k_reduce_pq(const double* __restrict__ partial, int nblk,
                                                   double* __restrict__ sc, int ipq, int iflag) {
  if (sc[iflag] != 0.0) return;
  __shared__ double sh[256];
  const double pq = block_sum256(partial, nblk, sh);
  if (threadIdx.x == 0) {
    sc[ipq] = pq;
    if (!(pq > 0.0) || !isfinite(pq)) sc[iflag] = 2.0;
  }
}

__global__ void __launch_bounds__(256) k_reduce_check(const double* __restrict__ partial, int nblk,
                                                      double* __restrict__ sc, int iiter, int nxt,
                                                      int irr, int iflag, int itol2) {
  if (sc[iflag] != 0.0) return;
  __shared__ double sh[256];
  const double rr = block_sum256(partial, nblk, sh);
  __syncthreads();
  const double rz = block_sum256(partial + nblk, nblk, sh);
  if (threadIdx.x == 0) {
    sc[iiter] += 1.0;
    sc[nxt] = rz;
    sc[irr] = rr;
    if (!isfinite(rr)) sc[iflag] = 2.0;
    else if (rr <= sc[itol2]) sc[iflag] = 1.0;
  }
}

__global__ void __launch_bounds__(256) k_cg_check_tail(double* __restrict__ sc, CgCheck ck,
                                                       const long long* __restrict__ sd) {
  if (sd) {   // batched: block z tests RVE z
    const long long d = sd[blockIdx.z];
    sc = at_slot(sc, d);
    ck.part = at_slot(ck.part, d);
  }
  if (sc[ck.iflag] != 0.0) return;
  __shared__ double red[8];
  double rz;
  (void)cg_check_inline(ck, sc, red, rz);
}

void launch_cg_check_tail(double* sc, const CgCheck& ck, hipStream_t st, const long long* sd,
                          int nslot) {
  hipLaunchKernelGGL(k_cg_check_tail, dim3(1, 1, nslot), dim3(256), 0, st, sc, ck, sd);
}

void launch_reduce_pq(const double* partial, int nblk, double* sc, int ipq, int iflag,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_pq, dim3(1), dim3(256), 0, st, partial, nblk, sc, ipq, iflag);
}
void launch_reduce_check(const double* partial, int nblk, double* sc, int iiter, int nxt, int irr,
                         int iflag, int itol2, hipStream_t st) {
  hipLaunchKernelGGL(k_reduce_check, dim3(1), dim3(256), 0, st, partial, nblk, sc, iiter, nxt,
                     irr, iflag, itol2);
}

__device__ __forceinline__ double pw_weight(long long b, const Grid& g) {
  const int kx = (int)(b % g.n1h);
  return (kx == 0 || (g.n1 % 2 == 0 && kx == g.n1 / 2)) ? 1.0 : 2.0;
}

template <typename R>
__global__ void __launch_bounds__(256) k_sdot(const cplx<R>* __restrict__ a, const cplx<R>* __restrict__ bv, long long cs,
                       int ncomp, Grid g, double* __restrict__ partial,
                       const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int c = 0; c < ncomp; ++c) {
      const cplx<R> x = a[c * cs + b], y = bv[c * cs + b];
      s += (double)x.x * (double)y.x + (double)x.y * (double)y.y;
    }
    acc += pw_weight(b, g) * s;
  }
  block_partial_sum(acc, partial, red);
}

template <typename R>
int launch_sdot(const Plans& p, const cplx<R>* a, const cplx<R>* b, long long cs, int ncomp,
                double* partial, hipStream_t st, const double* stop) {
  const int nb = vgrid(p.g.nspec);
  hipLaunchKernelGGL((k_sdot<R>), dim3(nb), dim3(256), 0, st, a, b, cs, ncomp, p.g, partial, stop);
  return nb;
}

template int launch_sdot<double>(const Plans&, const cplx<double>*, const cplx<double>*, long long,
                                 int, double*, hipStream_t, const double*);
template int launch_sdot<float>(const Plans&, const cplx<float>*, const cplx<float>*, long long,
                                int, double*, hipStream_t, const double*);

// ---- real vectors (phase field) -------------------------------------------------------
__global__ void __launch_bounds__(256) k_rdot(long long n, const double* __restrict__ a, const double* __restrict__ b,
                       double* __restrict__ partial, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += a[i] * b[i];
  block_partial_sum(acc, partial, red);
}

int launch_rdot(long long n, const double* a, const double* b, double* partial, hipStream_t st,
                const double* stop) {
  const int nb = vgrid(n);
  hipLaunchKernelGGL(k_rdot, dim3(nb), dim3(256), 0, st, n, a, b, partial, stop);
  return nb;
}

__global__ void __launch_bounds__(256) k_pf_pq(long long n, const double* __restrict__ p, const double* __restrict__ w,
                        const double* __restrict__ S, double* __restrict__ partial,
                        const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    acc += p[i] * (w[i] + 2.0 * S[i] * p[i]);
  block_partial_sum(acc, partial, red);
}

int launch_pf_pq(long long n, const double* p, const double* w, const double* S, double* partial,
                 hipStream_t st, const double* stop) {
  const int nb = vgrid(n);
  hipLaunchKernelGGL(k_pf_pq, dim3(nb), dim3(256), 0, st, n, p, w, S, partial, stop);
  return nb;
}

__global__ void __launch_bounds__(256) k_pf_xr(long long n, double* __restrict__ x, double* __restrict__ r,
                        const double* __restrict__ p, const double* __restrict__ w,
                        const double* __restrict__ S, const double* __restrict__ sc, int ia, int ib,
                        double* __restrict__ partial, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double red[16];
  const double al = sc[ia] / sc[ib];
  double acc = 0.0;
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double pp = p[i];
    x[i] += al * pp;
    const double rr = r[i] - al * (w[i] + 2.0 * S[i] * pp);
    r[i] = rr;
    acc += rr * rr;
  }
  block_partial_sum(acc, partial, red);
}

int launch_pf_xr(long long n, double* x, double* r, const double* p, const double* w,
                 const double* S, const double* sc, int ia, int ib, double* partial, hipStream_t st,
                 const double* stop) {
  const int nb = vgrid(n);
  hipLaunchKernelGGL(k_pf_xr, dim3(nb), dim3(256), 0, st, n, x, r, p, w, S, sc, ia, ib, partial,
                     stop);
  return nb;
}

__global__ void __launch_bounds__(256) k_pf_pw(long long n, double* __restrict__ p, double* __restrict__ w,
                        const double* __restrict__ z, const double* __restrict__ r,
                        const double* __restrict__ sc, int ia, int ib,
                        const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  const double be = sc[ia] / sc[ib];
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    p[i] = z[i] + be * p[i];
    w[i] = r[i] + be * w[i];
  }
}

void launch_pf_pw(long long n, double* p, double* w, const double* z, const double* r,
                  const double* sc, int ia, int ib, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL(k_pf_pw, dim3(vgrid(n)), dim3(256), 0, st, n, p, w, z, r, sc, ia, ib, stop);
}

__global__ void k_pf_check(double* __restrict__ sc, int iflag, int iiter, int ipq, int irr,
                           int itol2) {
  if (threadIdx.x != 0 || sc[iflag] != 0.0) return;
  sc[iiter] += 1.0;
  const double rr = sc[irr];
  if (!(sc[ipq] > 0.0) || !isfinite(rr)) sc[iflag] = 2.0;
  else if (rr <= sc[itol2]) sc[iflag] = 1.0;
}

void launch_pf_check(double* sc, int iflag, int iiter, int ipq, int irr, int itol2,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_pf_check, dim3(1), dim3(64), 0, st, sc, iflag, iiter, ipq, irr, itol2);
}

__global__ void __launch_bounds__(256) k_rscale(long long n, const double* __restrict__ x, double a, double* __restrict__ y) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    y[i] = a * x[i];
}

void launch_rscale(long long n, const double* x, double a, double* y, hipStream_t st) {
  hipLaunchKernelGGL(k_rscale, dim3(vgrid(n)), dim3(256), 0, st, n, x, a, y);
}

__global__ void __launch_bounds__(256) k_zero(uint32_t* __restrict__ p, long long nw) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < nw;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

void launch_zero(void* ptr, size_t bytes, hipStream_t st) {
  const long long nw = (long long)(bytes / 4);
  hipLaunchKernelGGL(k_zero, dim3(vgrid(nw)), dim3(256), 0, st, (uint32_t*)ptr, nw);
}

}  // namespace rvefft
