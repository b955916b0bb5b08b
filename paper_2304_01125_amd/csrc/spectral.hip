// FFT passes and pointwise Fourier-space operators (Sec. 3.1).
//
//  * x pass: real rows <-> half-spectrum rows (two rows packed per complex pencil);
//    the fused variant applies the degraded tangent g K : eps between the inverse
//    and the forward row transforms (the real-space part of the linearised
//    equilibrium operator of eq. newton);
//  * y / z passes: complex pencils along a strided axis, tiles of x-adjacent
//    pencils staged in LDS so that global accesses are contiguous along x;
//  * pointwise operators: symmetric gradient sym(i xi~ (x) u^) (eq. fdef),
//    divergence i xi~ . sigma^ (eq. momentum), the preconditioner
//    [xi~ . Kbar . xi~]^-1 (eqs. precf, avstiff), the phase-field scaling
//    (1 + l^2 |xi|^2)^-1 (eq. precph) and the regularised curl of the plastic
//    distortion (Nye tensor, eq. nye1 and its Fourier form).
// xi~ is xi with the Nyquist index of an even axis set to zero (odd derivatives
// of a real field); |xi|^2 keeps it.
#include "kernels.h"
#include "fft.h"

namespace rvefft {

static constexpr double kTwoPi = 6.283185307179586476925286766559;

__device__ __forceinline__ double freq(int k, int N, double L, bool tilde) {
  if (tilde && (N % 2 == 0) && k == N / 2) return 0.0;
  int m = (k <= (N - 1) / 2) ? k : k - N;
  return kTwoPi * (double)m / L;
}

template <typename R>
__device__ __forceinline__ void load_twiddles(cplx<R>* tw_s, const cplx<R>* tw_g, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) tw_s[t] = tw_g[t];
}

// ---------------------------------------------------------------------------
// x pass, real -> half spectrum.  Row r of the flattened (comp, k, j) order is
// voxel row rem = r % (N2*N3) of component c = r / (N2*N3).
template <typename R, typename TI>
__global__ void __launch_bounds__(256) k_x_r2c(const TI* __restrict__ in, long long in_cs, const double* __restrict__ phi,
                        double kres, cplx<R>* __restrict__ out, long long out_cs, int ncomp,
                        Grid g, AxisPlan pl, const cplx<R>* __restrict__ tw_g, int P) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.n1, NH = g.n1h, pitch = N + 1;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long rows_per_comp = (long long)g.n2 * g.n3;
  const long long nrows = rows_per_comp * ncomp;
  const long long pair0 = (long long)blockIdx.x * P;
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, i = t % N;
    const long long r0 = 2 * (pair0 + p), r1 = r0 + 1;
    R a = 0, b = 0;
    if (r0 < nrows) {
      const long long c = r0 / rows_per_comp, rem = r0 % rows_per_comp;
      const long long v = rem * N + i;
      double x = (double)in[c * in_cs + v];
      if (phi) { double q = 1.0 - phi[v]; x *= q * q + kres; }
      a = (R)x;
    }
    if (r1 < nrows) {
      const long long c = r1 / rows_per_comp, rem = r1 % rows_per_comp;
      const long long v = rem * N + i;
      double x = (double)in[c * in_cs + v];
      if (phi) { double q = 1.0 - phi[v]; x *= q * q + kres; }
      b = (R)x;
    }
    A[p * pitch + i] = cplx<R>{a, b};
  }
  __syncthreads();
  cplx<R>* Z = fft_pencils<R, false>(A, B, tw, pl, P, 1, pitch, false);
  for (int t = threadIdx.x; t < P * NH; t += blockDim.x) {
    const int p = t / NH, k = t % NH;
    const long long r0 = 2 * (pair0 + p), r1 = r0 + 1;
    if (r0 >= nrows) continue;
    const cplx<R> zk = Z[p * pitch + k];
    const cplx<R> zm = Z[p * pitch + ((N - k) % N)];
    // A_k = (Z_k + conj Z_-k)/2 ; B_k = (Z_k - conj Z_-k)/(2i)
    const cplx<R> ak = {R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    const cplx<R> bk = {R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
    {
      const long long c = r0 / rows_per_comp, rem = r0 % rows_per_comp;
      out[c * out_cs + rem * NH + k] = ak;
    }
    if (r1 < nrows) {
      const long long c = r1 / rows_per_comp, rem = r1 % rows_per_comp;
      out[c * out_cs + rem * NH + k] = bk;
    }
  }
}

// Half spectrum of row r at bin k, read as a Hermitian row: the imaginary parts of
// bin 0 and of the Nyquist bin are dropped (they do not exist for a real row).
template <typename R>
__device__ __forceinline__ cplx<R> herm_bin(const cplx<R>* row, int k, int N) {
  const int NH = N / 2 + 1;
  if (k < NH) {
    cplx<R> v = row[k];
    if (k == 0 || (N % 2 == 0 && k == N / 2)) v.y = 0;
    return v;
  }
  cplx<R> v = row[N - k];
  v.y = -v.y;
  return v;
}

// x pass, half spectrum -> real; out = scale * x (or out += scale * x).  When
// `track` is set, per-block maxima of |scale*x| and of |out - ref| are written to
// partial[0][blk] and partial[1][blk].
template <typename R, typename TO>
__global__ void __launch_bounds__(256) k_x_c2r(const cplx<R>* __restrict__ in, long long in_cs, TO* __restrict__ out,
                        long long out_cs, int ncomp, double scale, int accumulate, Grid g,
                        AxisPlan pl, const cplx<R>* __restrict__ tw_g, int P) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.n1, NH = g.n1h, pitch = N + 1;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long rows_per_comp = (long long)g.n2 * g.n3;
  const long long nrows = rows_per_comp * ncomp;
  const long long pair0 = (long long)blockIdx.x * P;
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, k = t % N;
    const long long r0 = 2 * (pair0 + p), r1 = r0 + 1;
    cplx<R> a = {0, 0}, b = {0, 0};
    if (r0 < nrows) {
      const long long c = r0 / rows_per_comp, rem = r0 % rows_per_comp;
      a = herm_bin(in + c * in_cs + rem * NH, k, N);
    }
    if (r1 < nrows) {
      const long long c = r1 / rows_per_comp, rem = r1 % rows_per_comp;
      b = herm_bin(in + c * in_cs + rem * NH, k, N);
    }
    A[p * pitch + k] = cplx<R>{a.x - b.y, a.y + b.x};     // a + i b
  }
  __syncthreads();
  cplx<R>* Z = fft_pencils<R, false>(A, B, tw, pl, P, 1, pitch, true);
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, i = t % N;
    const long long r0 = 2 * (pair0 + p), r1 = r0 + 1;
    if (r0 >= nrows) continue;
    const cplx<R> z = Z[p * pitch + i];
    {
      const long long c = r0 / rows_per_comp, rem = r0 % rows_per_comp;
      TO* o = out + c * out_cs + rem * N + i;
      const double v = scale * (double)z.x;
      *o = accumulate ? (TO)((double)*o + v) : (TO)v;
    }
    if (r1 < nrows) {
      const long long c = r1 / rows_per_comp, rem = r1 % rows_per_comp;
      TO* o = out + c * out_cs + rem * N + i;
      const double v = scale * (double)z.y;
      *o = accumulate ? (TO)((double)*o + v) : (TO)v;
    }
  }
}

// Fused x pass of the equilibrium operator on 6 components (in place):
//   eps = F_x^-1{.}, sigma = scale * gK : eps (Mandel), out = F_x{sigma}.
// One block holds Q voxel rows; components (xx,yy), (zz,yz), (xz,xy) share pencils.
template <typename R>
__global__ void __launch_bounds__(256) k_x_tangent(cplx<R>* __restrict__ data, long long cs, const R* __restrict__ gK,
                            double scale, Grid g, AxisPlan pl, const cplx<R>* __restrict__ tw_g,
                            int Q) {
  extern __shared__ unsigned char smem_raw[];
  const int N = g.n1, NH = g.n1h, pitch = N + 1;
  const int P = 3 * Q;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long nrows = (long long)g.n2 * g.n3;
  const long long row0 = (long long)blockIdx.x * Q;
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, k = t % N;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    cplx<R> a = {0, 0}, b = {0, 0};
    if (rem < nrows) {
      a = herm_bin(data + (2 * pair) * cs + rem * NH, k, N);
      b = herm_bin(data + (2 * pair + 1) * cs + rem * NH, k, N);
    }
    A[p * pitch + k] = cplx<R>{a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  cplx<R>* Z = fft_pencils<R, false>(A, B, tw, pl, P, 1, pitch, true);
  cplx<R>* W = (Z == A) ? B : A;
  const R s2 = (R)1.41421356237309504880;
  for (int t = threadIdx.x; t < Q * N; t += blockDim.x) {
    const int q = t / N, i = t % N;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const long long v = rem * N + i;
    const cplx<R> z0 = Z[(3 * q + 0) * pitch + i];
    const cplx<R> z1 = Z[(3 * q + 1) * pitch + i];
    const cplx<R> z2 = Z[(3 * q + 2) * pitch + i];
    // Mandel strain
    R e[6] = {z0.x, z0.y, z1.x, s2 * z1.y, s2 * z2.x, s2 * z2.y};
    R k21[21];
#pragma unroll
    for (int c = 0; c < 21; ++c) k21[c] = gK[(long long)c * g.nvox + v];
    R s[6];
    int idx = 0;
    R full[6][6];
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) { full[a][b] = k21[idx]; full[b][a] = k21[idx]; ++idx; }
#pragma unroll
    for (int a = 0; a < 6; ++a) {
      R acc = 0;
#pragma unroll
      for (int b = 0; b < 6; ++b) acc += full[a][b] * e[b];
      s[a] = acc * (R)scale;
    }
    const R is2 = (R)0.70710678118654752440;
    W[(3 * q + 0) * pitch + i] = cplx<R>{s[0], s[1]};
    W[(3 * q + 1) * pitch + i] = cplx<R>{s[2], is2 * s[3]};
    W[(3 * q + 2) * pitch + i] = cplx<R>{is2 * s[4], is2 * s[5]};
  }
  __syncthreads();
  cplx<R>* other = (W == A) ? B : A;
  cplx<R>* Y = fft_pencils<R, false>(W, other, tw, pl, P, 1, pitch, false);
  for (int t = threadIdx.x; t < P * NH; t += blockDim.x) {
    const int p = t / NH, k = t % NH;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const cplx<R> zk = Y[p * pitch + k];
    const cplx<R> zm = Y[p * pitch + ((N - k) % N)];
    data[(2 * pair) * cs + rem * NH + k] = cplx<R>{R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    data[(2 * pair + 1) * cs + rem * NH + k] =
        cplx<R>{R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
  }
}

// y (axis 1) or z (axis 2) pass, in place on ncomp components.  Block = (tile of
// TX x-bins) x (index along the remaining axis); blockIdx.y = component.
template <typename R>
__global__ void __launch_bounds__(256) k_fft_strided(cplx<R>* __restrict__ data, long long cs, int axis, int inv, Grid g,
                              AxisPlan pl, const cplx<R>* __restrict__ tw_g, int TX) {
  extern __shared__ unsigned char smem_raw[];
  const int N = pl.n;
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
  cplx<R>* Z = fft_pencils<R, true>(A, B, tw, pl, TX, TX, 1, inv != 0);
  for (int t = threadIdx.x; t < TX * N; t += blockDim.x) {
    const int n = t / TX, x = t % TX;
    if (x < w) d[n * stride_n + x] = Z[n * TX + x];
  }
}

// ---------------------------------------------------------------------------
// Pointwise operators.  Thread per half-spectrum bin.
struct Bin {
  int kx, ky, kz;
};
__device__ __forceinline__ Bin bin_of(long long e, const Grid& g) {
  Bin b;
  b.kx = (int)(e % g.n1h);
  long long r = e / g.n1h;
  b.ky = (int)(r % g.n2);
  b.kz = (int)(r / g.n2);
  return b;
}

// e = sym(i xi~ (x) u)  (3 -> 6 components)
template <typename R>
__global__ void __launch_bounds__(256) k_sym_grad(const cplx<R>* __restrict__ u, long long ucs, cplx<R>* __restrict__ e,
                           long long ecs, Grid g) {
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const R t1 = (R)freq(q.kx, g.n1, g.L1, true);
    const R t2 = (R)freq(q.ky, g.n2, g.L2, true);
    const R t3 = (R)freq(q.kz, g.n3, g.L3, true);
    const cplx<R> u1 = u[b], u2 = u[ucs + b], u3 = u[2 * ucs + b];
    // i * (a) = (-a.y, a.x)
    auto ic = [](R s, cplx<R> a) { return cplx<R>{-s * a.y, s * a.x}; };
    const R h = R(0.5);
    e[b] = ic(t1, u1);
    e[ecs + b] = ic(t2, u2);
    e[2 * ecs + b] = ic(t3, u3);
    cplx<R> yz = cadd(ic(t2, u3), ic(t3, u2));
    cplx<R> xz = cadd(ic(t1, u3), ic(t3, u1));
    cplx<R> xy = cadd(ic(t1, u2), ic(t2, u1));
    e[3 * ecs + b] = cscale(yz, h);
    e[4 * ecs + b] = cscale(xz, h);
    e[5 * ecs + b] = cscale(xy, h);
  }
}

// out = sign * i xi~ . s  (6 -> 3 components)
template <typename R>
__global__ void __launch_bounds__(256) k_div(const cplx<R>* __restrict__ s, long long scs, cplx<R>* __restrict__ out,
                      long long ocs, double sign, Grid g) {
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const R t1 = (R)freq(q.kx, g.n1, g.L1, true);
    const R t2 = (R)freq(q.ky, g.n2, g.L2, true);
    const R t3 = (R)freq(q.kz, g.n3, g.L3, true);
    const cplx<R> xx = s[b], yy = s[scs + b], zz = s[2 * scs + b];
    const cplx<R> yz = s[3 * scs + b], xz = s[4 * scs + b], xy = s[5 * scs + b];
    const R sg = (R)sign;
    cplx<R> d1 = {t1 * xx.x + t2 * xy.x + t3 * xz.x, t1 * xx.y + t2 * xy.y + t3 * xz.y};
    cplx<R> d2 = {t1 * xy.x + t2 * yy.x + t3 * yz.x, t1 * xy.y + t2 * yy.y + t3 * yz.y};
    cplx<R> d3 = {t1 * xz.x + t2 * yz.x + t3 * zz.x, t1 * xz.y + t2 * yz.y + t3 * zz.y};
    out[b] = cplx<R>{-sg * d1.y, sg * d1.x};
    out[ocs + b] = cplx<R>{-sg * d2.y, sg * d2.x};
    out[2 * ocs + b] = cplx<R>{-sg * d3.y, sg * d3.x};
  }
}

// Bin of -k on a self-conjugate x-plane (same kx, negated ky and kz).
__device__ __forceinline__ long long partner_bin(const Bin& q, const Grid& g) {
  const int ky = (g.n2 - q.ky) % g.n2, kz = (g.n3 - q.kz) % g.n3;
  return (long long)q.kx + (long long)g.n1h * (ky + (long long)g.n2 * kz);
}

// In-place projection of ncomp half-spectrum components onto spectra of real fields:
// on the x-planes kx = 0 and kx = N1/2 each pair (k, -k) is replaced by its Hermitian
// part.  One thread per bin of those planes; the thread of the smaller index of a
// pair writes both entries.
template <typename R>
__global__ void __launch_bounds__(256) k_herm_proj(cplx<R>* __restrict__ v, long long cs, int ncomp,
                                                   Grid g) {
  const int nplanes = (g.n1 % 2 == 0 && g.n1 > 1) ? 2 : 1;
  const long long per = (long long)g.n2 * g.n3;
  for (long long t = blockIdx.x * (long long)blockDim.x + threadIdx.x; t < per * nplanes;
       t += (long long)gridDim.x * blockDim.x) {
    Bin q;
    q.kx = (t < per) ? 0 : g.n1 / 2;
    const long long rem = t % per;
    q.ky = (int)(rem % g.n2);
    q.kz = (int)(rem / g.n2);
    const long long b = (long long)q.kx + (long long)g.n1h * rem;
    const long long bp = partner_bin(q, g);
    if (bp < b) continue;
    for (int c = 0; c < ncomp; ++c) {
      const cplx<R> a = v[c * cs + b], o = v[c * cs + bp];
      const cplx<R> h = {R(0.5) * (a.x + o.x), R(0.5) * (a.y - o.y)};
      v[c * cs + b] = h;
      v[c * cs + bp] = cplx<R>{h.x, -h.y};
    }
  }
}

template <typename R>
void launch_herm_proj(const Plans& p, cplx<R>* v, long long cs, int ncomp, hipStream_t st) {
  const long long n = (long long)p.g.n2 * p.g.n3 * 2;
  long long nb = (n + 255) / 256;
  hipLaunchKernelGGL((k_herm_proj<R>), dim3((int)(nb < 1 ? 1 : nb)), dim3(256), 0, st, v, cs,
                     ncomp, p.g);
}
template void launch_herm_proj<double>(const Plans&, cplx<double>*, long long, int, hipStream_t);
template void launch_herm_proj<float>(const Plans&, cplx<float>*, long long, int, hipStream_t);

// Mandel index of the symmetric pair (i, j) and its weight.
__device__ __forceinline__ int mandel_index(int i, int j) {
  if (i == j) return i;
  const int s = i + j;           // (1,2)->3 ; (0,2)->2 ; (0,1)->1
  return s == 3 ? 3 : (s == 2 ? 4 : 5);
}

// Parseval weight of a half-spectrum bin (x-bins 0 and N1/2 stand for themselves).
__device__ __forceinline__ double parseval_w(int kx, int n1) {
  return (kx == 0 || (n1 % 2 == 0 && kx == n1 / 2)) ? 1.0 : 2.0;
}

// z = M r with M = [xi~ . Kbar . xi~]^-1 (zero where xi~ = 0), and the block
// partial of the Parseval-weighted <r, z>.  kbar21 is the 21-entry Mandel mean
// tangent (device).
template <typename R>
__global__ void __launch_bounds__(256) k_precond(const cplx<R>* __restrict__ r, cplx<R>* __restrict__ z, long long cs,
                          const double* __restrict__ kbar21, Grid g, double* __restrict__ partial) {
  __shared__ double K4[81];
  __shared__ double red[1024 / 64];
  if (threadIdx.x < 81) {
    const int i = threadIdx.x / 27, j = (threadIdx.x / 9) % 3, k = (threadIdx.x / 3) % 3,
              l = threadIdx.x % 3;
    const int a = mandel_index(i, j), b = mandel_index(k, l);
    const int lo = min(a, b), hi = max(a, b);
    const int idx = lo * 6 - lo * (lo - 1) / 2 + (hi - lo);
    const double wa = (a < 3) ? 1.0 : 1.41421356237309504880;
    const double wb = (b < 3) ? 1.0 : 1.41421356237309504880;
    K4[threadIdx.x] = kbar21[idx] / (wa * wb);
  }
  __syncthreads();
  double acc = 0.0;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const double t[3] = {freq(q.kx, g.n1, g.L1, true), freq(q.ky, g.n2, g.L2, true),
                         freq(q.kz, g.n3, g.L3, true)};
    cplx<R> ri[3] = {r[b], r[cs + b], r[2 * cs + b]};
    if (q.kx == 0 || (g.n1 % 2 == 0 && q.kx == g.n1 / 2)) {
      // self-conjugate x-planes: keep the Hermitian part r(k) = conj r(-k) only
      const long long bp = partner_bin(q, g);
      for (int c = 0; c < 3; ++c) {
        const cplx<R> o = r[c * cs + bp];
        ri[c] = cplx<R>{R(0.5) * (ri[c].x + o.x), R(0.5) * (ri[c].y - o.y)};
      }
    }
    cplx<R> zo[3] = {{0, 0}, {0, 0}, {0, 0}};
    if (t[0] != 0.0 || t[1] != 0.0 || t[2] != 0.0) {
      double A[3][3];
      for (int i = 0; i < 3; ++i)
        for (int k = i; k < 3; ++k) {
          double s = 0.0;
          for (int j = 0; j < 3; ++j)
            for (int l = 0; l < 3; ++l) s += t[j] * K4[((i * 3 + j) * 3 + k) * 3 + l] * t[l];
          A[i][k] = s;
          A[k][i] = s;
        }
      const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
      const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
      const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
      const double det = A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02;
      const double id = 1.0 / det;
      double Mi[3][3];
      Mi[0][0] = c00 * id;
      Mi[0][1] = (A[0][2] * A[2][1] - A[0][1] * A[2][2]) * id;
      Mi[0][2] = (A[0][1] * A[1][2] - A[0][2] * A[1][1]) * id;
      Mi[1][1] = (A[0][0] * A[2][2] - A[0][2] * A[2][0]) * id;
      Mi[1][2] = (A[0][2] * A[1][0] - A[0][0] * A[1][2]) * id;
      Mi[2][2] = (A[0][0] * A[1][1] - A[0][1] * A[1][0]) * id;
      Mi[1][0] = Mi[0][1];
      Mi[2][0] = Mi[0][2];
      Mi[2][1] = Mi[1][2];
      for (int i = 0; i < 3; ++i) {
        double zx = 0, zy = 0;
        for (int k = 0; k < 3; ++k) { zx += Mi[i][k] * (double)ri[k].x; zy += Mi[i][k] * (double)ri[k].y; }
        zo[i] = cplx<R>{(R)zx, (R)zy};
      }
    }
    z[b] = zo[0];
    z[cs + b] = zo[1];
    z[2 * cs + b] = zo[2];
    const double w = parseval_w(q.kx, g.n1);
    double d = 0.0;
    for (int i = 0; i < 3; ++i) d += (double)ri[i].x * (double)zo[i].x + (double)ri[i].y * (double)zo[i].y;
    acc += w * d;
  }
  block_partial_sum(acc, partial, red);
}

// d *= scale / (1 + l^2 |xi|^2)  (1 component)
template <typename R>
__global__ void __launch_bounds__(256) k_pf_scale(cplx<R>* __restrict__ d, double ell, double scale, Grid g) {
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const double x1 = freq(q.kx, g.n1, g.L1, false), x2 = freq(q.ky, g.n2, g.L2, false),
                 x3 = freq(q.kz, g.n3, g.L3, false);
    const double s = scale / (1.0 + ell * ell * (x1 * x1 + x2 * x2 + x3 * x3));
    const cplx<R> v = d[b];
    d[b] = cplx<R>{(R)(s * (double)v.x), (R)(s * (double)v.y)};
  }
}

// Regularised Nye tensor in Fourier space, in place on 9 components (row-major
// beta_il): Lambda_ij = sum_kl eps_jkl i xi~_k beta~_il with
// beta~ = beta / (1 + l_fp^2 |xi|^2), times `scale`.
template <typename R>
__global__ void __launch_bounds__(256) k_curl_reg(cplx<R>* __restrict__ b9, long long cs, double ell_fp, double scale,
                           Grid g) {
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const double x1 = freq(q.kx, g.n1, g.L1, false), x2 = freq(q.ky, g.n2, g.L2, false),
                 x3 = freq(q.kz, g.n3, g.L3, false);
    const double reg = scale / (1.0 + ell_fp * ell_fp * (x1 * x1 + x2 * x2 + x3 * x3));
    const double t[3] = {freq(q.kx, g.n1, g.L1, true), freq(q.ky, g.n2, g.L2, true),
                         freq(q.kz, g.n3, g.L3, true)};
    for (int i = 0; i < 3; ++i) {
      double bx[3], by[3];
      for (int l = 0; l < 3; ++l) {
        const cplx<R> v = b9[(3 * i + l) * cs + b];
        bx[l] = reg * (double)v.x;
        by[l] = reg * (double)v.y;
      }
      // (xi~ x beta_i.)_j = eps_jkl xi~_k beta_il ; then multiply by i
      const double cx[3] = {t[1] * bx[2] - t[2] * bx[1], t[2] * bx[0] - t[0] * bx[2],
                            t[0] * bx[1] - t[1] * bx[0]};
      const double cy[3] = {t[1] * by[2] - t[2] * by[1], t[2] * by[0] - t[0] * by[2],
                            t[0] * by[1] - t[1] * by[0]};
      for (int j = 0; j < 3; ++j) b9[(3 * i + j) * cs + b] = cplx<R>{(R)(-cy[j]), (R)cx[j]};
    }
  }
}

// ---------------------------------------------------------------------------
// Host launchers.
static size_t xpass_smem(int n1, int P, size_t csz) { return ((size_t)n1 + (size_t)P * (n1 + 1) * 2) * csz; }

template <typename R>
static int pick_rows(int n1, size_t budget, int maxP) {
  int P = maxP;
  while (P > 1 && xpass_smem(n1, P, sizeof(cplx<R>)) > budget) P /= 2;
  return P;
}

static constexpr size_t kLdsBudget = 64 * 1024;

template <typename R>
void launch_x_r2c(const Plans& p, const void* in, bool in_f64, long long in_cs, const double* phi,
                  double kres, cplx<R>* out, long long out_cs, int ncomp, hipStream_t st) {
  const Grid& g = p.g;
  const int P = pick_rows<R>(g.n1, kLdsBudget, 16);
  const long long pairs = ((long long)g.n2 * g.n3 * ncomp + 1) / 2;
  const int nblk = (int)((pairs + P - 1) / P);
  const size_t sm = xpass_smem(g.n1, P, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  if (in_f64)
    hipLaunchKernelGGL((k_x_r2c<R, double>), dim3(nblk), dim3(256), sm, st, (const double*)in,
                       in_cs, phi, kres, out, out_cs, ncomp, g, p.ax[0], tw, P);
  else
    hipLaunchKernelGGL((k_x_r2c<R, float>), dim3(nblk), dim3(256), sm, st, (const float*)in, in_cs,
                       phi, kres, out, out_cs, ncomp, g, p.ax[0], tw, P);
}

template <typename R>
void launch_x_c2r(const Plans& p, const cplx<R>* in, long long in_cs, void* out, bool out_f64,
                  long long out_cs, int ncomp, double scale, int accumulate, hipStream_t st) {
  const Grid& g = p.g;
  const int P = pick_rows<R>(g.n1, kLdsBudget, 16);
  const long long pairs = ((long long)g.n2 * g.n3 * ncomp + 1) / 2;
  const int nblk = (int)((pairs + P - 1) / P);
  const size_t sm = xpass_smem(g.n1, P, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  if (out_f64)
    hipLaunchKernelGGL((k_x_c2r<R, double>), dim3(nblk), dim3(256), sm, st, in, in_cs,
                       (double*)out, out_cs, ncomp, scale, accumulate, g, p.ax[0], tw, P);
  else
    hipLaunchKernelGGL((k_x_c2r<R, float>), dim3(nblk), dim3(256), sm, st, in, in_cs,
                       (float*)out, out_cs, ncomp, scale, accumulate, g, p.ax[0], tw, P);
}

template <typename R>
void launch_x_tangent(const Plans& p, cplx<R>* data, long long cs, const R* gK, double scale,
                      hipStream_t st) {
  const Grid& g = p.g;
  int Q = 8;
  while (Q > 1 && xpass_smem(g.n1, 3 * Q, sizeof(cplx<R>)) > kLdsBudget) Q /= 2;
  const long long rows = (long long)g.n2 * g.n3;
  const int nblk = (int)((rows + Q - 1) / Q);
  const size_t sm = xpass_smem(g.n1, 3 * Q, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  hipLaunchKernelGGL((k_x_tangent<R>), dim3(nblk), dim3(256), sm, st, data, cs, gK, scale, g,
                     p.ax[0], tw, Q);
}

template <typename R>
void launch_fft_yz(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis, bool inv,
                   hipStream_t st) {
  const Grid& g = p.g;
  const AxisPlan& pl = p.ax[axis];
  const int N = pl.n;
  int TX = 16;
  while (TX > 1 && ((size_t)N + 2 * (size_t)TX * N) * sizeof(cplx<R>) > kLdsBudget) TX /= 2;
  const int ntiles = (g.n1h + TX - 1) / TX;
  const int others = (axis == 1) ? g.n3 : g.n2;
  const size_t sm = ((size_t)N + 2 * (size_t)TX * N) * sizeof(cplx<R>);
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(axis, sizeof(R) == 8);
  hipLaunchKernelGGL((k_fft_strided<R>), dim3(ntiles * others, ncomp), dim3(256), sm, st, data, cs,
                     axis, inv ? 1 : 0, g, pl, tw, TX);
}

static int grid_for(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

template <typename R>
void launch_sym_grad(const Plans& p, const cplx<R>* u, long long ucs, cplx<R>* e, long long ecs,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_sym_grad<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, u, ucs, e, ecs,
                     p.g);
}

template <typename R>
void launch_div(const Plans& p, const cplx<R>* s, long long scs, cplx<R>* out, long long ocs,
                double sign, hipStream_t st) {
  hipLaunchKernelGGL((k_div<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, s, scs, out, ocs,
                     sign, p.g);
}

template <typename R>
int launch_precond(const Plans& p, const cplx<R>* r, cplx<R>* z, long long cs, const double* kbar21,
                   double* partial, hipStream_t st) {
  const int nb = grid_for(p.g.nspec);
  hipLaunchKernelGGL((k_precond<R>), dim3(nb), dim3(256), 0, st, r, z, cs, kbar21, p.g, partial);
  return nb;
}

template <typename R>
void launch_pf_scale(const Plans& p, cplx<R>* d, double ell, double scale, hipStream_t st) {
  hipLaunchKernelGGL((k_pf_scale<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, d, ell, scale,
                     p.g);
}

template <typename R>
void launch_curl_reg(const Plans& p, cplx<R>* b9, long long cs, double ell_fp, double scale,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_curl_reg<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, b9, cs, ell_fp,
                     scale, p.g);
}

#define RVE_INST(R)                                                                              \
  template void launch_x_r2c<R>(const Plans&, const void*, bool, long long, const double*, double, \
                                cplx<R>*, long long, int, hipStream_t);                          \
  template void launch_x_c2r<R>(const Plans&, const cplx<R>*, long long, void*, bool, long long,  \
                                int, double, int, hipStream_t);                                  \
  template void launch_x_tangent<R>(const Plans&, cplx<R>*, long long, const R*, double,          \
                                    hipStream_t);                                                \
  template void launch_fft_yz<R>(const Plans&, cplx<R>*, long long, int, int, bool, hipStream_t); \
  template void launch_sym_grad<R>(const Plans&, const cplx<R>*, long long, cplx<R>*, long long,  \
                                   hipStream_t);                                                 \
  template void launch_div<R>(const Plans&, const cplx<R>*, long long, cplx<R>*, long long,       \
                              double, hipStream_t);                                              \
  template int launch_precond<R>(const Plans&, const cplx<R>*, cplx<R>*, long long,               \
                                 const double*, double*, hipStream_t);                           \
  template void launch_pf_scale<R>(const Plans&, cplx<R>*, double, double, hipStream_t);          \
  template void launch_curl_reg<R>(const Plans&, cplx<R>*, long long, double, double, hipStream_t);

RVE_INST(double)
RVE_INST(float)

}  // namespace rvefft
