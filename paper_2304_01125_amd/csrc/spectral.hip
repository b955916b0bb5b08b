// Pointwise Fourier-space operators (Sec. 3.1): symmetric gradient sym(i xi~ (x) u^) (eq. fdef),
//    divergence i xi~ . sigma^ (eq. momentum), the preconditioner
//    [xi~ . Kbar . xi~]^-1 (eqs. precf, avstiff), the phase-field scaling
//    (1 + l^2 |xi|^2)^-1 (eq. precph) and the regularised curl of the plastic
//    distortion (Nye tensor, eq. nye1 and its Fourier form).
// xi~ is xi with the Nyquist index of an even axis set to zero (odd derivatives
// of a real field); |xi|^2 keeps it.
#include "kernels.h"

#include <algorithm>

namespace rvefft {


static int grid_for(long long n);

// ---------------------------------------------------------------------------
// Pointwise operators.  Thread per half-spectrum bin.
struct Bin {
  int kx, ky, kz;
};
// (32-bit unsigned division: a half spectrum has fewer than 2^32 bins)
__device__ __forceinline__ Bin bin_of(long long e, const Grid& g) {
  Bin b;
  const unsigned u = (unsigned)e, n1h = (unsigned)g.n1h, n2 = (unsigned)g.n2;
  const unsigned r = u / n1h;
  b.kx = (int)(u - r * n1h);
  const unsigned kz = r / n2;
  b.ky = (int)(r - kz * n2);
  b.kz = (int)kz;
  return b;
}

// General derivative symbols k (kvec): e = sym(k (x) u), and sum_j c_j s_ij with c =
// conj(k) (the adjoint of the gradient) for the divergence-type operators.
template <typename R>
__device__ __forceinline__ void sym_grad_k(const cplx<double> k[3], const cplx<R> u[3],
                                           cplx<R> e[6]) {
  cplx<double> ud[3];
  for (int c = 0; c < 3; ++c) ud[c] = cplx<double>{(double)u[c].x, (double)u[c].y};
  auto cv = [](cplx<double> a) { return cplx<R>{(R)a.x, (R)a.y}; };
  e[0] = cv(cmul(k[0], ud[0]));
  e[1] = cv(cmul(k[1], ud[1]));
  e[2] = cv(cmul(k[2], ud[2]));
  e[3] = cv(cscale(cadd(cmul(k[1], ud[2]), cmul(k[2], ud[1])), 0.5));
  e[4] = cv(cscale(cadd(cmul(k[0], ud[2]), cmul(k[2], ud[0])), 0.5));
  e[5] = cv(cscale(cadd(cmul(k[0], ud[1]), cmul(k[1], ud[0])), 0.5));
}
template <typename R>
__device__ __forceinline__ void adj_div_k(const cplx<double> k[3], const cplx<R> sg[6],
                                          cplx<double> d[3]) {
  // stress components xx yy zz yz xz xy; row i of sigma: (i, x), (i, y), (i, z)
  constexpr int row[3][3] = {{0, 5, 4}, {5, 1, 3}, {4, 3, 2}};
  for (int i = 0; i < 3; ++i) {
    cplx<double> a{0.0, 0.0};
    for (int j = 0; j < 3; ++j) {
      const cplx<R> v = sg[row[i][j]];
      a = cadd(a, cmul(cconj(k[j]), cplx<double>{(double)v.x, (double)v.y}));
    }
    d[i] = a;
  }
}

// e = sym(i xi~ (x) u)  (3 -> 6 components)
template <typename R>
__global__ void __launch_bounds__(256) k_sym_grad(const cplx<R>* __restrict__ u, long long ucs, cplx<R>* __restrict__ e,
                           long long ecs, Grid g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    if (g.sch) {
      cplx<double> k[3];
      kvec(g, q.kx, q.ky, q.kz, k);
      const cplx<R> uu[3] = {u[b], u[ucs + b], u[2 * ucs + b]};
      cplx<R> ee[6];
      sym_grad_k(k, uu, ee);
      for (int c = 0; c < 6; ++c) e[c * ecs + b] = ee[c];
      continue;
    }
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
                      long long ocs, double sign, Grid g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    if (g.sch) {      // out = -sign conj(k) . s (= sign i xi~ . s for the spectral symbol)
      cplx<double> k[3], d[3];
      kvec(g, q.kx, q.ky, q.kz, k);
      const cplx<R> sg6[6] = {s[b], s[scs + b], s[2 * scs + b], s[3 * scs + b], s[4 * scs + b],
                              s[5 * scs + b]};
      adj_div_k(k, sg6, d);
      for (int c = 0; c < 3; ++c) out[c * ocs + b] = cplx<R>{(R)(-sign * d[c].x), (R)(-sign * d[c].y)};
      continue;
    }
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
                                                   Grid g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
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
void launch_herm_proj(const Plans& p, cplx<R>* v, long long cs, int ncomp, hipStream_t st,
                      const double* stop) {
  const long long n = (long long)p.g.n2 * p.g.n3 * 2;
  long long nb = (n + 255) / 256;
  hipLaunchKernelGGL((k_herm_proj<R>), dim3((int)(nb < 1 ? 1 : nb)), dim3(256), 0, st, v, cs,
                     ncomp, p.g, stop);
}
template void launch_herm_proj<double>(const Plans&, cplx<double>*, long long, int, hipStream_t,
                                       const double*);
template void launch_herm_proj<float>(const Plans&, cplx<float>*, long long, int, hipStream_t,
                                      const double*);

// Mandel index of the symmetric pair (i, j) and its weight.
__device__ __forceinline__ int mandel_index(int i, int j) {
  if (i == j) return i;
  const int s = i + j;           // (1,2)->3 ; (0,2)->2 ; (0,1)->1
  return s == 3 ? 3 : (s == 2 ? 4 : 5);
}


// Fourth-order mean tangent from its 21 Mandel entries into LDS (81 values).
__device__ __forceinline__ void load_kbar4(double* K4, const double* __restrict__ kbar21) {
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
}

// The acoustic tensor A_ik = sum_jl t_j K_ijkl t_l as 6 x 6 coefficients on the products
// tau = (t0 t0, t1 t1, t2 t2, t1 t2, t0 t2, t0 t1): A_p = sum_m C[p][m] tau_m for the pairs
// p = (i, k) in 00 01 02 11 12 22, with C = K_ijkl for j = l and K_ijkl + K_ilkj for
// m = (j, l), j < l.  36 uniform values (LDS), 36 FMA per bin.
__device__ __forceinline__ double kbar_entry(const double* __restrict__ kbar21, int i, int j,
                                             int k, int l) {
  const int a = mandel_index(i, j), b = mandel_index(k, l);
  const int lo = min(a, b), hi = max(a, b);
  const int idx = lo * 6 - lo * (lo - 1) / 2 + (hi - lo);
  const double wa = (a < 3) ? 1.0 : 1.41421356237309504880;
  const double wb = (b < 3) ? 1.0 : 1.41421356237309504880;
  return kbar21[idx] / (wa * wb);
}
__device__ __forceinline__ void load_acoustic36(double* C, const double* __restrict__ kbar21) {
  if (threadIdx.x < 36) {
    constexpr int pi[6] = {0, 0, 0, 1, 1, 2}, pk[6] = {0, 1, 2, 1, 2, 2};
    constexpr int mj[6] = {0, 1, 2, 1, 0, 0}, ml[6] = {0, 1, 2, 2, 2, 1};
    const int p = threadIdx.x / 6, m = threadIdx.x % 6;
    const int i = pi[p], k = pk[p], j = mj[m], l = ml[m];
    double c = kbar_entry(kbar21, i, j, k, l);
    if (j != l) c += kbar_entry(kbar21, i, l, k, j);
    C[threadIdx.x] = c;
  }
}

// Zero bin under mixed macroscopic control: zo = m0 ri on the bin's six reals
// (Mandel macro components xx, yy, zz, yz, xz, xy held as x: (xx, xy), y: (yy, yz),
// z: (zz, xz)).
template <typename R>
__device__ __forceinline__ void apply_M0(const double* __restrict__ m0, const cplx<R> ri[3],
                                         cplx<R> zo[3]) {
  const double rm[6] = {(double)ri[0].x, (double)ri[1].x, (double)ri[2].x,
                        (double)ri[1].y, (double)ri[2].y, (double)ri[0].y};
  double zm[6];
  for (int i = 0; i < 6; ++i) {
    double a = 0.0;
    for (int j = 0; j < 6; ++j) a += m0[i * 6 + j] * rm[j];
    zm[i] = a;
  }
  zo[0] = cplx<R>{(R)zm[0], (R)zm[5]};
  zo[1] = cplx<R>{(R)zm[1], (R)zm[3]};
  zo[2] = cplx<R>{(R)zm[2], (R)zm[4]};
}

// ro = F zi on the zero bin's six reals (as apply_M0), in FP64
template <typename R>
__device__ __forceinline__ void apply_F0(const double* __restrict__ f, const cplx<R> zi[3],
                                         cplx<double> ro[3]) {
  const double zm[6] = {(double)zi[0].x, (double)zi[1].x, (double)zi[2].x,
                        (double)zi[1].y, (double)zi[2].y, (double)zi[0].y};
  double rm[6];
  for (int i = 0; i < 6; ++i) {
    double a = 0.0;
    for (int j = 0; j < 6; ++j) a += f[i * 6 + j] * zm[j];
    rm[i] = a;
  }
  ro[0] = cplx<double>{rm[0], rm[5]};
  ro[1] = cplx<double>{rm[1], rm[3]};
  ro[2] = cplx<double>{rm[2], rm[4]};
}

// zo = [t . K . t]^-1 ri (zero where t = 0), t = xi~ of the bin, the acoustic tensor from
// the 36 coefficients of load_acoustic36; with As set, the acoustic tensor t . K . t itself
// (upper triangle: 00 01 02 11 12 22; zero where t = 0).
template <typename R>
__device__ __forceinline__ void apply_M6(const double t[3], const double* C, const cplx<R> ri[3],
                                         cplx<R> zo[3], double* As = nullptr) {
  zo[0] = zo[1] = zo[2] = cplx<R>{0, 0};
  if (As)
    for (int i = 0; i < 6; ++i) As[i] = 0.0;
  if (t[0] == 0.0 && t[1] == 0.0 && t[2] == 0.0) return;
  const double tau[6] = {t[0] * t[0], t[1] * t[1], t[2] * t[2], t[1] * t[2], t[0] * t[2],
                         t[0] * t[1]};
  double a6[6];
#pragma unroll
  for (int p = 0; p < 6; ++p) {
    double s = 0.0;
#pragma unroll
    for (int m = 0; m < 6; ++m) s += C[p * 6 + m] * tau[m];
    a6[p] = s;
  }
  if (As)
    for (int i = 0; i < 6; ++i) As[i] = a6[i];
  const double A[3][3] = {{a6[0], a6[1], a6[2]}, {a6[1], a6[3], a6[4]}, {a6[2], a6[4], a6[5]}};
  const double c00 = A[1][1] * A[2][2] - A[1][2] * A[2][1];
  const double c01 = A[1][2] * A[2][0] - A[1][0] * A[2][2];
  const double c02 = A[1][0] * A[2][1] - A[1][1] * A[2][0];
  const double id = 1.0 / (A[0][0] * c00 + A[0][1] * c01 + A[0][2] * c02);
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

// zo = [conj(k) . K . k]^-1 ri (zero where k = 0): the Hermitian acoustic tensor of the
// general derivative symbol, inverted by its adjugate.
template <typename R>
__device__ __forceinline__ void apply_Mk(const cplx<double> k[3], const double* K4,
                                         const cplx<R> ri[3], cplx<R> zo[3],
                                         cplx<double>* Ah = nullptr) {
  zo[0] = zo[1] = zo[2] = cplx<R>{0, 0};
  if (Ah)
    for (int i = 0; i < 6; ++i) Ah[i] = cplx<double>{0.0, 0.0};
  if (k[0].x == 0.0 && k[0].y == 0.0 && k[1].x == 0.0 && k[1].y == 0.0 && k[2].x == 0.0 &&
      k[2].y == 0.0)
    return;
  // W_jl = conj(k_j) k_l (Hermitian), then the upper triangle of A_im = K_ijml W_jl
  cplx<double> W[3][3];
  for (int j = 0; j < 3; ++j)
    for (int l = j; l < 3; ++l) {
      W[j][l] = cmul(cconj(k[j]), k[l]);
      W[l][j] = cconj(W[j][l]);
    }
  cplx<double> A[3][3];
  for (int i = 0; i < 3; ++i)
    for (int m = i; m < 3; ++m) {
      double sr = 0.0, si = 0.0;
      for (int j = 0; j < 3; ++j)
        for (int l = 0; l < 3; ++l) {
          const double kv = K4[((i * 3 + j) * 3 + m) * 3 + l];
          sr += kv * W[j][l].x;
          si += kv * W[j][l].y;
        }
      A[i][m] = cplx<double>{sr, si};
      A[m][i] = cplx<double>{sr, -si};
    }
  if (Ah) {
    Ah[0] = A[0][0]; Ah[1] = A[0][1]; Ah[2] = A[0][2];
    Ah[3] = A[1][1]; Ah[4] = A[1][2]; Ah[5] = A[2][2];
  }
  auto c = [&](int i0, int j0, int i1, int j1) {   // A[i0][j0] A[i1][j1] - A[i0][j1] A[i1][j0]
    return csub(cmul(A[i0][j0], A[i1][j1]), cmul(A[i0][j1], A[i1][j0]));
  };
  cplx<double> adj[3][3];
  adj[0][0] = c(1, 1, 2, 2); adj[0][1] = c(0, 2, 2, 1); adj[0][2] = c(0, 1, 1, 2);
  adj[1][0] = c(1, 2, 2, 0); adj[1][1] = c(0, 0, 2, 2); adj[1][2] = c(0, 2, 1, 0);
  adj[2][0] = c(1, 0, 2, 1); adj[2][1] = c(0, 1, 2, 0); adj[2][2] = c(0, 0, 1, 1);
  const cplx<double> det = cadd(cadd(cmul(A[0][0], adj[0][0]), cmul(A[0][1], adj[1][0])),
                                cmul(A[0][2], adj[2][0]));
  const double dd = det.x * det.x + det.y * det.y;
  const cplx<double> idet{det.x / dd, -det.y / dd};
  for (int i = 0; i < 3; ++i) {
    cplx<double> z{0.0, 0.0};
    for (int m = 0; m < 3; ++m)
      z = cadd(z, cmul(adj[i][m], cplx<double>{(double)ri[m].x, (double)ri[m].y}));
    z = cmul(z, idet);
    zo[i] = cplx<R>{(R)z.x, (R)z.y};
  }
}

// ---- fused conjugate-gradient kernels ---------------------------------------------
// p = z + beta p (beta = sc[ia] / sc[ib]), then e = sym(i xi~ (x) p)  (3 -> 6 comps).
template <typename R>
__global__ void __launch_bounds__(256)
k_grad_cgp(cplx<R>* __restrict__ pv, const cplx<R>* __restrict__ z, long long cs,
           const double* __restrict__ sc, int ia, int ib, cplx<R>* __restrict__ e, long long ecs,
           Grid g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  const double be = sc[ia] / sc[ib];
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const R t1 = (R)freq(q.kx, g.n1, g.L1, true);
    const R t2 = (R)freq(q.ky, g.n2, g.L2, true);
    const R t3 = (R)freq(q.kz, g.n3, g.L3, true);
    cplx<R> u[3];
    for (int c = 0; c < 3; ++c) {
      const cplx<R> zz = z[c * cs + b], pp = pv[c * cs + b];
      u[c] = cplx<R>{(R)((double)zz.x + be * (double)pp.x), (R)((double)zz.y + be * (double)pp.y)};
      pv[c * cs + b] = u[c];
    }
    if (g.sch) {
      cplx<double> k[3];
      kvec(g, q.kx, q.ky, q.kz, k);
      cplx<R> ee[6];
      sym_grad_k(k, u, ee);
      for (int c = 0; c < 6; ++c) e[c * ecs + b] = ee[c];
      continue;
    }
    auto ic = [](R s, cplx<R> a) { return cplx<R>{-s * a.y, s * a.x}; };
    const R h = R(0.5);
    e[b] = ic(t1, u[0]);
    e[ecs + b] = ic(t2, u[1]);
    e[2 * ecs + b] = ic(t3, u[2]);
    e[3 * ecs + b] = cscale(cadd(ic(t2, u[2]), ic(t3, u[1])), h);
    e[4 * ecs + b] = cscale(cadd(ic(t1, u[2]), ic(t3, u[0])), h);
    e[5 * ecs + b] = cscale(cadd(ic(t1, u[1]), ic(t2, u[0])), h);
  }
}

// q = -i xi~ . s  (6 -> 3 comps) and the block partial of the Parseval-weighted <p, q>.
template <typename R>
__global__ void __launch_bounds__(256)
k_div_dot(const cplx<R>* __restrict__ s, long long scs, cplx<R>* __restrict__ out, long long ocs,
          const cplx<R>* __restrict__ pv, Grid g, double* __restrict__ partial,
          const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double red[16];
  double acc = 0.0;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    if (g.sch) {      // q = conj(k) . s
      cplx<double> k[3], dd[3];
      kvec(g, q.kx, q.ky, q.kz, k);
      const cplx<R> sg6[6] = {s[b], s[scs + b], s[2 * scs + b], s[3 * scs + b], s[4 * scs + b],
                              s[5 * scs + b]};
      adj_div_k(k, sg6, dd);
      double dot = 0.0;
      for (int c = 0; c < 3; ++c) {
        const cplx<R> qq = {(R)dd[c].x, (R)dd[c].y};
        out[c * ocs + b] = qq;
        const cplx<R> pp = pv[c * ocs + b];
        dot += (double)pp.x * (double)qq.x + (double)pp.y * (double)qq.y;
      }
      acc += parseval_w(q.kx, g.n1) * dot;
      continue;
    }
    const R t1 = (R)freq(q.kx, g.n1, g.L1, true);
    const R t2 = (R)freq(q.ky, g.n2, g.L2, true);
    const R t3 = (R)freq(q.kz, g.n3, g.L3, true);
    const cplx<R> xx = s[b], yy = s[scs + b], zz = s[2 * scs + b];
    const cplx<R> yz = s[3 * scs + b], xz = s[4 * scs + b], xy = s[5 * scs + b];
    const cplx<R> d[3] = {
        {t1 * xx.x + t2 * xy.x + t3 * xz.x, t1 * xx.y + t2 * xy.y + t3 * xz.y},
        {t1 * xy.x + t2 * yy.x + t3 * yz.x, t1 * xy.y + t2 * yy.y + t3 * yz.y},
        {t1 * xz.x + t2 * yz.x + t3 * zz.x, t1 * xz.y + t2 * yz.y + t3 * zz.y}};
    double dot = 0.0;
    for (int c = 0; c < 3; ++c) {
      const cplx<R> qq = {d[c].y, -d[c].x};        // -i d
      out[c * ocs + b] = qq;
      const cplx<R> pp = pv[c * ocs + b];
      dot += (double)pp.x * (double)qq.x + (double)pp.y * (double)qq.y;
    }
    acc += parseval_w(q.kx, g.n1) * dot;
  }
  block_partial_sum(acc, partial, red);
}

template <typename R>
void launch_grad_cgp(const Plans& p, cplx<R>* pv, const cplx<R>* z, long long cs, const double* sc,
                     int ia, int ib, cplx<R>* e, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_grad_cgp<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, pv, z, cs, sc,
                     ia, ib, e, cs, p.g, stop);
}
template <typename R>
int launch_div_dot(const Plans& p, const cplx<R>* s, cplx<R>* q, const cplx<R>* pv, long long cs,
                   double* partial, hipStream_t st, const double* stop) {
  const int nb = grid_for(p.g.nspec);
  hipLaunchKernelGGL((k_div_dot<R>), dim3(nb), dim3(256), 0, st, s, cs, q, cs, pv, p.g, partial,
                     stop);
  return nb;
}

// One CG step (see launch_cg_step in kernels.h); SCH: derivative symbol of the
// preconditioner (0 spectral, 1 rotated).
template <typename R, int SCH>
__global__ void __launch_bounds__(256)
k_cg_step(cplx<R>* __restrict__ x, const cplx<R>* __restrict__ pv,
          const cplx<R>* __restrict__ qv, cplx<R>* __restrict__ z, long long cs,
          const double* __restrict__ kbar21, double* __restrict__ sc, int cur, int ipq,
          Grid g, double* __restrict__ partial, const double* __restrict__ stop,
          const double* __restrict__ pq_part, int nb_pq, int iflag, int iiter,
          const double* __restrict__ m0) {
  {
    const long long d = slot_delta(g);
    x = at_slot(x, d); pv = at_slot(pv, d); qv = at_slot(qv, d); z = at_slot(z, d);
    kbar21 = at_slot(kbar21, d); sc = at_slot(sc, d); partial = at_slot(partial, d);
    stop = at_slot(stop, d); pq_part = at_slot(pq_part, d); m0 = at_slot(m0, d);
  }
  if (stop && *stop != 0.0) return;
  __shared__ double K4[81];
  __shared__ double red[16];
  double pq;
  if (pq_part) {
    pq = block_sum_all(pq_part, nb_pq, red);
    const bool bad = !(pq > 0.0) || !isfinite(pq);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      sc[ipq] = pq;
      if (bad) sc[iflag] = 2.0;
      else sc[iiter] += 1.0;
    }
    if (bad) return;
  } else {
    pq = sc[ipq];
  }
  if constexpr (SCH == 0) load_acoustic36(K4, kbar21);
  else load_kbar4(K4, kbar21);
  __syncthreads();
  const double al = sc[cur] / pq;
  const bool even = (g.n1 % 2 == 0);
  double rr = 0.0, rz = 0.0;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    cplx<R> pl[3], ql[3], xl[3], zl[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      // streamed: x is touched here only, once per iteration; streaming p and q as well
      // measured faster for the passes that follow
      const long long i = c * cs + b;
      pl[c] = ld_stream(pv + i);
      ql[c] = ld_stream(qv + i);
      xl[c] = ld_stream(x + i);
      zl[c] = z[i];
    }
    const Bin q = bin_of(b, g);
    const double t[3] = {freq(q.kx, g.n1, g.L1, true), freq(q.ky, g.n2, g.L2, true),
                         freq(q.kz, g.n3, g.L3, true)};
    const bool mac = m0 && b == 0;           // macro unknowns: no projection, z = m0 r
    const bool selfconj = !mac && ((q.kx == 0) || (even && q.kx == g.n1 / 2));
    const long long bp = selfconj ? partner_bin(q, g) : b;
    cplx<R> hq[3], mq[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      const long long i = c * cs + b;
      const cplx<R> pp = pl[c];
      cplx<R> qq = ql[c];
      if (selfconj) {
        const cplx<R> qo = qv[c * cs + bp];
        qq = cplx<R>{R(0.5) * (qq.x + qo.x), R(0.5) * (qq.y - qo.y)};
      }
      hq[c] = qq;
      cplx<R> xx = xl[c];
      xx.x = (R)((double)xx.x + al * (double)pp.x);
      xx.y = (R)((double)xx.y + al * (double)pp.y);
      st_stream(x + i, xx);
    }
    // an offset the compiler cannot see through: it would otherwise hoist the 81
    // loop-invariant K4 reads out of the loop into registers (169 VGPRs, two waves per
    // SIMD); LDS reads per bin cost less than the lost occupancy
    int koff = 0;
    asm volatile("" : "+v"(koff));
    const double* K4b = K4 + koff;
    // z -= alpha M h(q) (M is per bin, so z = M r stays exact without storing r), then
    // r = M^-1 z from the same per-bin tensor for <r, r> and <r, z>
    cplx<R> zn[3];
    cplx<double> rd[3];
    auto z_update = [&]() {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        zn[c] = cplx<R>{(R)((double)zl[c].x - al * (double)mq[c].x),
                        (R)((double)zl[c].y - al * (double)mq[c].y)};
        z[c * cs + b] = zn[c];
      }
    };
    if (mac) {
      apply_M0(m0, hq, mq);
      z_update();
      apply_F0(m0 + 36, zn, rd);
    } else if constexpr (SCH == 0) {
      double As[6];
      apply_M6(t, K4b, hq, mq, As);
      z_update();
      const double A[3][3] = {{As[0], As[1], As[2]}, {As[1], As[3], As[4]},
                              {As[2], As[4], As[5]}};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        double rx = 0.0, ry = 0.0;
#pragma unroll
        for (int m = 0; m < 3; ++m) {
          rx += A[i][m] * (double)zn[m].x;
          ry += A[i][m] * (double)zn[m].y;
        }
        rd[i] = cplx<double>{rx, ry};
      }
    } else {
      cplx<double> kk[3], Ah[6];
      kvec(g, q.kx, q.ky, q.kz, kk);
      apply_Mk(kk, K4b, hq, mq, Ah);
      z_update();
      const cplx<double> A[3][3] = {{Ah[0], Ah[1], Ah[2]},
                                    {cconj(Ah[1]), Ah[3], Ah[4]},
                                    {cconj(Ah[2]), cconj(Ah[4]), Ah[5]}};
#pragma unroll
      for (int i = 0; i < 3; ++i) {
        cplx<double> acc{0.0, 0.0};
#pragma unroll
        for (int m = 0; m < 3; ++m)
          acc = cadd(acc, cmul(A[i][m], cplx<double>{(double)zn[m].x, (double)zn[m].y}));
        rd[i] = acc;
      }
    }
    double a = 0.0, bz = 0.0;
    for (int c = 0; c < 3; ++c) {
      a += rd[c].x * rd[c].x + rd[c].y * rd[c].y;
      bz += rd[c].x * (double)zn[c].x + rd[c].y * (double)zn[c].y;
    }
    const double w = parseval_w(q.kx, g.n1);
    rr += w * a;
    rz += w * bz;
  }
  for (int off = 32; off > 0; off >>= 1) {
    rr += __shfl_down(rr, off, 64);
    rz += __shfl_down(rz, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) { red[wid] = rr; red[8 + wid] = rz; }
  __syncthreads();
  if (threadIdx.x < 2) {
    double sum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += red[8 * threadIdx.x + w];
    partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] = sum;
  }
}

template <typename R>
int launch_cg_step(const Plans& p, cplx<R>* x, const cplx<R>* pv, const cplx<R>* q,
                   cplx<R>* z, long long cs, const double* kbar21, double* sc, int cur, int ipq,
                   double* partial, hipStream_t st, const double* stop, const double* pq_part,
                   int nb_pq, int iflag, int iiter, int max_blocks, const double* m0) {
  const int nb = std::min(grid_for(p.g.nspec), max_blocks);
  if (p.g.sch)
    hipLaunchKernelGGL((k_cg_step<R, 1>), dim3(nb, 1, p.nslot), dim3(256), 0, st, x, pv, q, z, cs, kbar21,
                       sc, cur, ipq, p.g, partial, stop, pq_part, nb_pq, iflag, iiter, m0);
  else
    hipLaunchKernelGGL((k_cg_step<R, 0>), dim3(nb, 1, p.nslot), dim3(256), 0, st, x, pv, q, z, cs, kbar21,
                       sc, cur, ipq, p.g, partial, stop, pq_part, nb_pq, iflag, iiter, m0);
  return nb;
}
template int launch_cg_step<double>(const Plans&, cplx<double>*,
                                    const cplx<double>*, const cplx<double>*, cplx<double>*,
                                    long long, const double*, double*, int, int, double*,
                                    hipStream_t, const double*, const double*, int, int, int,
                                    int, const double*);
template int launch_cg_step<float>(const Plans&, cplx<float>*, const cplx<float>*,
                                   const cplx<float>*, cplx<float>*, long long, const double*,
                                   double*, int, int, double*, hipStream_t, const double*,
                                   const double*, int, int, int, int, const double*);
#define RVE_CG_INST(R)                                                                           \
  template void launch_grad_cgp<R>(const Plans&, cplx<R>*, const cplx<R>*, long long,             \
                                   const double*, int, int, cplx<R>*, hipStream_t, const double*); \
  template int launch_div_dot<R>(const Plans&, const cplx<R>*, cplx<R>*, const cplx<R>*,          \
                                 long long, double*, hipStream_t, const double*);

RVE_CG_INST(double)
RVE_CG_INST(float)

// z = M r with M = [xi~ . Kbar . xi~]^-1 (zero where xi~ = 0), and the block
// partial of the Parseval-weighted <r, z>.  kbar21 is the 21-entry Mandel mean
// tangent (device).
template <typename R>
__global__ void __launch_bounds__(256) k_precond(const cplx<R>* __restrict__ r, cplx<R>* __restrict__ z, long long cs,
                          const double* __restrict__ kbar21, Grid g, double* __restrict__ partial,
                          const double* __restrict__ stop, const double* __restrict__ m0) {
  if (stop && *stop != 0.0) return;
  __shared__ double K4[81];
  __shared__ double C36[36];
  __shared__ double red[1024 / 64];
  load_acoustic36(C36, kbar21);
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
    const bool mac = m0 && b == 0;           // macro unknowns: no projection, z = m0 r
    if (!mac && (q.kx == 0 || (g.n1 % 2 == 0 && q.kx == g.n1 / 2))) {
      // self-conjugate x-planes: keep the Hermitian part r(k) = conj r(-k) only
      const long long bp = partner_bin(q, g);
      for (int c = 0; c < 3; ++c) {
        const cplx<R> o = r[c * cs + bp];
        ri[c] = cplx<R>{R(0.5) * (ri[c].x + o.x), R(0.5) * (ri[c].y - o.y)};
      }
    }
    cplx<R> zo[3] = {{0, 0}, {0, 0}, {0, 0}};
    int koff = 0;                            // keeps the K4 reads in the loop, see k_cg_step
    asm volatile("" : "+v"(koff));
    const double* K4b = K4 + koff;
    if (mac) {
      apply_M0(m0, ri, zo);
    } else if (g.sch) {
      cplx<double> kk[3];
      kvec(g, q.kx, q.ky, q.kz, kk);
      apply_Mk(kk, K4b, ri, zo);
    } else {
      apply_M6(t, C36 + koff, ri, zo);
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
// d *= scale / (1 + l^2 |xi|^2) (lap = 0: the phase-field preconditioner), or
// d *= scale l^2 |xi|^2 (lap = 1: the operator -l^2 lap)
__global__ void __launch_bounds__(256) k_pf_scale(cplx<R>* __restrict__ d, double ell, double scale, Grid g,
                                                  const double* __restrict__ stop, int lap) {
  if (stop && *stop != 0.0) return;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const Bin q = bin_of(b, g);
    const double x1 = freq(q.kx, g.n1, g.L1, false), x2 = freq(q.ky, g.n2, g.L2, false),
                 x3 = freq(q.kz, g.n3, g.L3, false);
    const double l2x2 = ell * ell * (x1 * x1 + x2 * x2 + x3 * x3);
    const double s = lap ? scale * l2x2 : scale / (1.0 + l2x2);
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
static int grid_for(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

template <typename R>
void launch_sym_grad(const Plans& p, const cplx<R>* u, long long ucs, cplx<R>* e, long long ecs,
                     hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_sym_grad<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, u, ucs, e, ecs,
                     p.g, stop);
}

template <typename R>
void launch_div(const Plans& p, const cplx<R>* s, long long scs, cplx<R>* out, long long ocs,
                double sign, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_div<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, s, scs, out, ocs,
                     sign, p.g, stop);
}

template <typename R>
int launch_precond(const Plans& p, const cplx<R>* r, cplx<R>* z, long long cs, const double* kbar21,
                   double* partial, hipStream_t st, const double* stop, const double* m0) {
  const int nb = grid_for(p.g.nspec);
  hipLaunchKernelGGL((k_precond<R>), dim3(nb), dim3(256), 0, st, r, z, cs, kbar21, p.g, partial,
                     stop, m0);
  return nb;
}

template <typename R>
void launch_pf_scale(const Plans& p, cplx<R>* d, double ell, double scale, hipStream_t st,
                     const double* stop, int lap) {
  hipLaunchKernelGGL((k_pf_scale<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, d, ell, scale,
                     p.g, stop, lap);
}

template <typename R>
void launch_curl_reg(const Plans& p, cplx<R>* b9, long long cs, double ell_fp, double scale,
                     hipStream_t st) {
  hipLaunchKernelGGL((k_curl_reg<R>), dim3(grid_for(p.g.nspec)), dim3(256), 0, st, b9, cs, ell_fp,
                     scale, p.g);
}

#define RVE_INST(R)                                                                              \
  template void launch_sym_grad<R>(const Plans&, const cplx<R>*, long long, cplx<R>*, long long,  \
                                   hipStream_t, const double*);                                  \
  template void launch_div<R>(const Plans&, const cplx<R>*, long long, cplx<R>*, long long,       \
                              double, hipStream_t, const double*);                               \
  template int launch_precond<R>(const Plans&, const cplx<R>*, cplx<R>*, long long,               \
                                 const double*, double*, hipStream_t, const double*,             \
                                 const double*);                                                 \
  template void launch_pf_scale<R>(const Plans&, cplx<R>*, double, double, hipStream_t,          \
                                   const double*, int);                                          \
  template void launch_curl_reg<R>(const Plans&, cplx<R>*, long long, double, double, hipStream_t);

RVE_INST(double)
RVE_INST(float)

}  // namespace rvefft
