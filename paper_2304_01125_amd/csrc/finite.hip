// Finite-strain kinematics of the fatigue increment (Sec. 2.1: F = Fe Fp with the plastic
// velocity gradient Lp = sum_a gdot_a s_a (x) n_a; Sec. 3.1, eqs. str1, momentum, fdef,
// newton, precf, avstiff with the 9-component displacement gradient; eq. decMiehe with the
// logarithmic elastic strain).
//
// Return map: backward Euler on the plastic deformation with the strength frozen over the
// step, in the form of Kalidindi, Bronkhorst and Anand (1992).  With the trial elastic
// right Cauchy-Green tensor A = Fe*^T Fe*, Fe* = F Fp_n^-1, the second Piola-Kirchhoff
// stress S of the lattice configuration is the root of
//     C^-1 (S - S*) + sum_a dgamma_a(S : Q_a) Q_a = 0,   S* = C 1/2 (A - I),
//     Q_a = sym(A s_a (x) n_a)   (tau_a = S : Q_a: the Mandel stress of the trial state),
// the gradient of a strictly convex potential (the small-strain one with the Schmid
// tensors P_a replaced by Q_a): Newton with backtracking on it, in the crystal frame.
// Then Fp = (I + sum_a dgamma_a s_a (x) n_a) Fp_n and P = F Fp^-1 S Fp^-T; the 9 x 9
// consistent tangent dP/dF follows by differentiating every step (the root condition
// implicitly: dS = K_S (1/2 dA - sum_a [dgamma_a' (S : dQ_a) Q_a + dgamma_a dQ_a]),
// K_S = (C^-1 + sum_a dgamma_a' Q_a Q_a^T)^-1).
//
// Tensors of 9 components are row-major (F_ij at 3 i + j), fields structure-of-arrays;
// the tangent is stored as gK[(9 r + c) N + v] = g(phi) dP_r / dF_c.
#include "cpdev.h"

namespace rvefft {

namespace {

// ---- 3 x 3 algebra (row-major) ----------------------------------------------------------
__device__ __forceinline__ void mm3(const double* a, const double* b, double* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[j] + a[3 * i + 1] * b[3 + j] + a[3 * i + 2] * b[6 + j];
}
// c = a^T b
__device__ __forceinline__ void mtm3(const double* a, const double* b, double* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) c[3 * i + j] = a[i] * b[j] + a[3 + i] * b[3 + j] + a[6 + i] * b[6 + j];
}
// c = a b^T
__device__ __forceinline__ void mmt3(const double* a, const double* b, double* c) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j)
      c[3 * i + j] = a[3 * i] * b[3 * j] + a[3 * i + 1] * b[3 * j + 1] + a[3 * i + 2] * b[3 * j + 2];
}
// general inverse by the adjugate; false if singular
__device__ __forceinline__ bool inv3(const double* a, double* ai) {
  const double c00 = a[4] * a[8] - a[5] * a[7], c01 = a[5] * a[6] - a[3] * a[8],
               c02 = a[3] * a[7] - a[4] * a[6];
  const double det = a[0] * c00 + a[1] * c01 + a[2] * c02;
  if (!(det != 0.0) || !isfinite(det)) return false;
  const double id = 1.0 / det;
  ai[0] = c00 * id;
  ai[1] = (a[2] * a[7] - a[1] * a[8]) * id;
  ai[2] = (a[1] * a[5] - a[2] * a[4]) * id;
  ai[3] = c01 * id;
  ai[4] = (a[0] * a[8] - a[2] * a[6]) * id;
  ai[5] = (a[2] * a[3] - a[0] * a[5]) * id;
  ai[6] = c02 * id;
  ai[7] = (a[1] * a[6] - a[0] * a[7]) * id;
  ai[8] = (a[0] * a[4] - a[1] * a[3]) * id;
  return true;
}
// crystal components R^T T R of a sample-frame tensor (R: crystal -> sample)
__device__ __forceinline__ void to_cry(const double* R, const double* T, double* o) {
  double W[9];
  mm3(T, R, W);
  mtm3(R, W, o);
}
// sample components R T R^T of a crystal-frame tensor
__device__ __forceinline__ void to_smp(const double* R, const double* T, double* o) {
  double W[9];
  mmt3(T, R, W);
  mm3(R, W, o);
}
// Mandel vector of sym(T) (order xx yy zz yz xz xy, sqrt 2 on the shears)
__device__ __forceinline__ void mandel_sym(const double* T, double m[6]) {
  m[0] = T[0];
  m[1] = T[4];
  m[2] = T[8];
  m[3] = kInvSqrt2 * (T[5] + T[7]);
  m[4] = kInvSqrt2 * (T[2] + T[6]);
  m[5] = kInvSqrt2 * (T[1] + T[3]);
}
__device__ __forceinline__ void from_mandel9(const double m[6], double* T) {
  T[0] = m[0];
  T[4] = m[1];
  T[8] = m[2];
  T[5] = T[7] = kInvSqrt2 * m[3];
  T[2] = T[6] = kInvSqrt2 * m[4];
  T[1] = T[3] = kInvSqrt2 * m[5];
}
// q = Mandel(sym((A s) (x) n)) for one slip system (A symmetric)
__device__ __forceinline__ void qdir(const double* A, const double* s, const double* n, double q[6]) {
  const double a0 = A[0] * s[0] + A[1] * s[1] + A[2] * s[2];
  const double a1 = A[3] * s[0] + A[4] * s[1] + A[5] * s[2];
  const double a2 = A[6] * s[0] + A[7] * s[1] + A[8] * s[2];
  q[0] = a0 * n[0];
  q[1] = a1 * n[1];
  q[2] = a2 * n[2];
  q[3] = kInvSqrt2 * (a1 * n[2] + a2 * n[1]);
  q[4] = kInvSqrt2 * (a0 * n[2] + a2 * n[0]);
  q[5] = kInvSqrt2 * (a0 * n[1] + a1 * n[0]);
}
__device__ __forceinline__ double dot6(const double* a, const double* b) {
  return a[0] * b[0] + a[1] * b[1] + a[2] * b[2] + a[3] * b[3] + a[4] * b[4] + a[5] * b[5];
}

// Potential of the finite-strain return map (crystal frame, directions from A)
template <int FL>
__device__ double fs_potential(const FsFrame& fr, const double* A, const double sig[6],
                               const double str[6], const Flow& f) {
  double d[6], Sd[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) d[i] = sig[i] - str[i];
  cubic_mul(fr.s11, fr.s12, fr.s66, d, Sd);
  const double el = dot6(d, Sd);
  double pl = 0.0;
#pragma unroll 1
  for (int a = 0; a < 12; ++a) {
    double q[6];
    qdir(A, fr.s + 3 * a, fr.n + 3 * a, q);
    pl += slip_pot<FL>(f, dot6(q, sig));
  }
  return 0.5 * el + pot_scale<FL>(f) * pl;
}

template <int FL>
__device__ void fs_resjac(const FsFrame& fr, const double* A, const double sig[6],
                          const double str[6], const Flow& f, double Rv[6], double J[21]) {
  double d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) d[i] = sig[i] - str[i];
  cubic_mul(fr.s11, fr.s12, fr.s66, d, Rv);
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j)
      J[pk(i, j)] = (i == j) ? (i < 3 ? fr.s11 : fr.s66) : ((j < 3) ? fr.s12 : 0.0);
#pragma unroll 1
  for (int a = 0; a < 12; ++a) {
    double q[6];
    qdir(A, fr.s + 3 * a, fr.n + 3 * a, q);
    double dg, ddg;
    slip_law<FL>(f, dot6(q, sig), dg, ddg);
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      Rv[i] += dg * q[i];
      const double di = ddg * q[i];
#pragma unroll
      for (int j = i; j < 6; ++j) J[pk(i, j)] += di * q[j];
    }
  }
}

// Newton with backtracking on the potential (as the small-strain return map); sig holds
// the warm start.  Returns the iteration count, or -1.
template <int FL>
__device__ int fs_return_map(const FsFrame& fr, const double* A, const double str[6],
                             const Flow& f, double sig[6]) {
  // start from the warm start or from the trial stress scaled into the elastic range,
  // whichever has the lower potential
  {
    double tmax = 0.0;
#pragma unroll 1
    for (int a = 0; a < 12; ++a) {
      double q[6];
      qdir(A, fr.s + 3 * a, fr.n + 3 * a, q);
      tmax = fmax(tmax, fabs(dot6(q, str)));
    }
    const double sc = fmin(1.0, 1.0 / fmax(tmax * f.ig, 1e-300));
    double sd[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) sd[i] = sc * str[i];
    const double pw = fs_potential<FL>(fr, A, sig, str, f);
    const double pd = fs_potential<FL>(fr, A, sd, str, f);
    if (!(pw <= pd)) {
#pragma unroll
      for (int i = 0; i < 6; ++i) sig[i] = sd[i];
    }
  }
  double scale = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) scale = fmax(scale, fabs(str[i]));
  scale += f.g;
  int it;
  bool conv = false;
  for (it = 0; it < 400; ++it) {
    double Rv[6], J[21], d[6], mR[6];
    fs_resjac<FL>(fr, A, sig, str, f, Rv, J);
    if (!chol6p(J)) return -1;
#pragma unroll
    for (int i = 0; i < 6; ++i) mR[i] = -Rv[i];
    chol6p_solve(J, mR, d);
    const double phi0 = fs_potential<FL>(fr, A, sig, str, f);
    const double slope = dot6(Rv, d);
    double t = 1.0;
    for (int ls = 0; ls < 60; ++ls) {
      double c[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) c[i] = sig[i] + t * d[i];
      const double phi1 = fs_potential<FL>(fr, A, c, str, f);
      if (phi1 <= phi0 + 1e-4 * t * slope + 1e-13 * fabs(phi0)) break;
      t *= 0.5;
    }
    double smax = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      const double st = t * d[i];
      sig[i] += st;
      smax = fmax(smax, fabs(st));
    }
    if (smax <= 1e-13 * scale) { conv = true; break; }
  }
  if (!conv) return -1;
  {   // one polishing Newton step at the root
    double Rv[6], J[21], d[6];
    fs_resjac<FL>(fr, A, sig, str, f, Rv, J);
    if (!chol6p(J)) return -1;
    chol6p_solve(J, Rv, d);
#pragma unroll
    for (int i = 0; i < 6; ++i) sig[i] -= d[i];
  }
  return it + 1;
}

__device__ __forceinline__ void load9(const double* __restrict__ f, long long N, long long v,
                                      double o[9]) {
#pragma unroll
  for (int c = 0; c < 9; ++c) o[c] = f[c * N + v];
}

// ---------------------------------------------------------------------------------------
// Constitutive update at F + t dF (dF may be null).  Writes the effective first
// Piola-Kirchhoff stress P (9), the trial plastic deformation Fp (9), g(phi) dP/dF (81),
// aux = (sum tau dgamma, sum |dgamma|, dLp : dLp, W_e+) and the crystal-frame S (6, the
// next call's warm start).  One voxel per thread.
template <int FL>
__global__ void __launch_bounds__(64)
k_fs_constitutive(long long N, const double* __restrict__ Fd, const double* __restrict__ dF,
                  double t, const double* __restrict__ Fpn, const double* __restrict__ gslip,
                  const int* __restrict__ grain, const double* __restrict__ gtab,
                  double* __restrict__ Sws, const double* __restrict__ phi, double* __restrict__ Pout,
                  double* __restrict__ fp_tr, double* __restrict__ aux, double* __restrict__ gK,
                  FsFrame fr, Material m, int* __restrict__ fail) {
  const long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x;
  if (v >= N) return;
  double F[9], Fpi[9], Fe[9], A[9], Ac[9], R[9];
  load9(Fd, N, v, F);
  if (dF) {
#pragma unroll
    for (int c = 0; c < 9; ++c) F[c] += t * dF[c * N + v];
  }
  {
    double Fp[9];
    load9(Fpn, N, v, Fp);
    if (!inv3(Fp, Fpi)) { atomicAdd(fail, 1); return; }
  }
  const double* Rg = gtab + (long long)grain[v] * GT_STRIDE + GT_R;
#pragma unroll
  for (int c = 0; c < 9; ++c) R[c] = Rg[c];
  mm3(F, Fpi, Fe);
  mtm3(Fe, Fe, A);
  to_cry(R, A, Ac);
  // trial: S* = C 1/2 (A - I) (crystal frame, Mandel)
  double e6[6], str[6], sig[6];
  {
    double E[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) E[c] = 0.5 * (Ac[c] - ((c % 4 == 0) ? 1.0 : 0.0));
    mandel_sym(E, e6);
  }
  cubic_mul(fr.c11, fr.c12, fr.c66, e6, str);
#pragma unroll
  for (int i = 0; i < 6; ++i) sig[i] = Sws[i * N + v];
  const double g = gslip[v];
  const Flow f = make_flow(m, g);
  if (fs_return_map<FL>(fr, Ac, str, f, sig) < 0) {
    atomicAdd(fail, 1);
#pragma unroll
    for (int i = 0; i < 6; ++i) sig[i] = str[i];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i) Sws[i * N + v] = sig[i];
  // slip, its derivative and the plastic velocity gradient increment (crystal frame)
  double dg[12], ddg[12], Lc[9];
  double dw = 0.0, sabs = 0.0;
#pragma unroll
  for (int c = 0; c < 9; ++c) Lc[c] = 0.0;
#pragma unroll 1
  for (int a = 0; a < 12; ++a) {
    double q[6];
    qdir(Ac, fr.s + 3 * a, fr.n + 3 * a, q);
    const double tau = dot6(q, sig);
    slip_law<FL>(f, tau, dg[a], ddg[a]);
    dw += tau * dg[a];
    sabs += fabs(dg[a]);
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) Lc[3 * i + j] += dg[a] * fr.s[3 * a + i] * fr.n[3 * a + j];
  }
  double dLp2 = 0.0;
#pragma unroll
  for (int c = 0; c < 9; ++c) dLp2 += Lc[c] * Lc[c];
  // K_S = (C^-1 + sum ddg q q^T)^-1 at the root
  double KS[21];
  {
    double Rv[6], J[21];
    fs_resjac<FL>(fr, Ac, sig, str, f, Rv, J);
    if (!chol6p(J)) {
      atomicAdd(fail, 1);
      return;
    }
    chol6p_inverse(J, KS);
  }
  // Fp = X Fp_n, X = I + dLp (sample frame); Gi = Fp^-1 = Fp_n^-1 X^-1
  double X[9], Xi[9], Gi[9], S[9];
  to_smp(R, Lc, X);
  X[0] += 1.0; X[4] += 1.0; X[8] += 1.0;
  if (!inv3(X, Xi)) { atomicAdd(fail, 1); return; }
  mm3(Fpi, Xi, Gi);
  {
    double Fp[9], Fpnew[9];
    load9(Fpn, N, v, Fp);
    mm3(X, Fp, Fpnew);
#pragma unroll
    for (int c = 0; c < 9; ++c) fp_tr[c * N + v] = Fpnew[c];
    double Sc[9];
    from_mandel9(sig, Sc);
    to_smp(R, Sc, S);
  }
  double FGi[9], Z[9], T1[9], Wm[9], P[9];
  mm3(F, Gi, FGi);          // Fe
  mmt3(S, Gi, Z);           // S Gi^T
  mm3(Gi, Z, T1);           // Gi S Gi^T
  mm3(FGi, S, Wm);          // F Gi S
  mm3(FGi, Z, P);           // F Gi S Gi^T
#pragma unroll
  for (int c = 0; c < 9; ++c) Pout[c * N + v] = P[c];
  // tensile elastic energy of the log strain (eq. decMiehe): eigenpairs of Ce = Fe^T Fe
  double wep;
  {
    double Ce[9];
    mtm3(FGi, FGi, Ce);
    double a3[3][3] = {{Ce[0], Ce[1], Ce[2]}, {Ce[3], Ce[4], Ce[5]}, {Ce[6], Ce[7], Ce[8]}};
    double d[3], V[3][3];
    jacobi3(a3, d, V);
    double Ep[9];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < 3; ++k) s += fmax(0.5 * log(d[k]), 0.0) * V[i][k] * V[j][k];
        Ep[3 * i + j] = s;
      }
    double Epc[9], em[6], cm[6];
    to_cry(R, Ep, Epc);
    mandel_sym(Epc, em);
    cubic_mul(fr.c11, fr.c12, fr.c66, em, cm);
    wep = 0.5 * dot6(em, cm);
  }
  aux[v] = dw;
  aux[N + v] = sabs;
  aux[2 * N + v] = dLp2;
  aux[3 * N + v] = wep;
  // consistent tangent, column by column
  const double ph = phi ? phi[v] : 0.0;
  const double gphi = (1.0 - ph) * (1.0 - ph) + m.kres;
#pragma unroll 1
  for (int k = 0; k < 3; ++k)
#pragma unroll 1
    for (int l = 0; l < 3; ++l) {
      double dA[9], dAc[9];
#pragma unroll
      for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
          dA[3 * a + b] = Fe[3 * k + a] * Fpi[3 * l + b] + Fe[3 * k + b] * Fpi[3 * l + a];
      to_cry(R, dA, dAc);
      double rhs[6], sdq[12];
      mandel_sym(dAc, rhs);
#pragma unroll
      for (int i = 0; i < 6; ++i) rhs[i] *= 0.5;
#pragma unroll 1
      for (int a = 0; a < 12; ++a) {
        double q[6], dq[6];
        qdir(Ac, fr.s + 3 * a, fr.n + 3 * a, q);
        qdir(dAc, fr.s + 3 * a, fr.n + 3 * a, dq);
        sdq[a] = dot6(sig, dq);
        const double cq = ddg[a] * sdq[a];
#pragma unroll
        for (int i = 0; i < 6; ++i) rhs[i] -= cq * q[i] + dg[a] * dq[i];
      }
      double dS6[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) {
        double s = 0.0;
#pragma unroll
        for (int j = 0; j < 6; ++j) s += KS[pk(i, j)] * rhs[j];
        dS6[i] = s;
      }
      double dLc[9];
#pragma unroll
      for (int c = 0; c < 9; ++c) dLc[c] = 0.0;
#pragma unroll 1
      for (int a = 0; a < 12; ++a) {
        double q[6];
        qdir(Ac, fr.s + 3 * a, fr.n + 3 * a, q);
        const double dd = ddg[a] * (dot6(dS6, q) + sdq[a]);
#pragma unroll
        for (int i = 0; i < 3; ++i)
#pragma unroll
          for (int j = 0; j < 3; ++j) dLc[3 * i + j] += dd * fr.s[3 * a + i] * fr.n[3 * a + j];
      }
      double dL[9], tmp[9], dGi[9], dSc[9], dS[9];
      to_smp(R, dLc, dL);
      mm3(Gi, dL, tmp);
      mm3(tmp, Xi, dGi);
#pragma unroll
      for (int c = 0; c < 9; ++c) dGi[c] = -dGi[c];
      from_mandel9(dS6, dSc);
      to_smp(R, dSc, dS);
      // dP = dF T1 + F dGi Z + Wm dGi^T + FGi dS Gi^T, dF = e_k (x) e_l
      double dP[9], a1[9], a2[9], a3[9], a4[9];
      mm3(F, dGi, a1);
      mm3(a1, Z, a2);
      mmt3(Wm, dGi, a3);
      mmt3(dS, Gi, a1);
      mm3(FGi, a1, a4);
#pragma unroll
      for (int c = 0; c < 9; ++c) dP[c] = a2[c] + a3[c] + a4[c];
#pragma unroll
      for (int j = 0; j < 3; ++j) dP[3 * k + j] += T1[3 * l + j];
      const int col = 3 * k + l;
#pragma unroll
      for (int r = 0; r < 9; ++r) gK[(long long)(9 * r + col) * N + v] = gphi * dP[r];
    }
}

// ---- pointwise Fourier operators on the half spectrum ------------------------------------
struct FsBin {
  int kx, ky, kz;
};
__device__ __forceinline__ FsBin fs_bin(long long e, const Grid& g) {
  FsBin b;
  const unsigned u = (unsigned)e, n1h = (unsigned)g.n1h, n2 = (unsigned)g.n2;
  const unsigned r = u / n1h;
  b.kx = (int)(u - r * n1h);
  const unsigned kz = r / n2;
  b.ky = (int)(r - kz * n2);
  b.kz = (int)kz;
  return b;
}

// e_ij = i xi~_j u_i (eq. fdef, 3 -> 9 components)
template <typename R>
__global__ void __launch_bounds__(256) k_fs_grad(const cplx<R>* __restrict__ u, long long ucs,
                                                 cplx<R>* __restrict__ e, long long ecs, Grid g,
                                                 const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const FsBin q = fs_bin(b, g);
    const R t[3] = {(R)freq(q.kx, g.n1, g.L1, true), (R)freq(q.ky, g.n2, g.L2, true),
                    (R)freq(q.kz, g.n3, g.L3, true)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      const cplx<R> ui = u[i * ucs + b];
#pragma unroll
      for (int j = 0; j < 3; ++j) e[(3 * i + j) * ecs + b] = cplx<R>{-t[j] * ui.y, t[j] * ui.x};
    }
  }
}

// out_i = sign i xi~_j s_ij  (9 -> 3 components)
template <typename R>
__global__ void __launch_bounds__(256) k_fs_div(const cplx<R>* __restrict__ s, long long scs,
                                                cplx<R>* __restrict__ out, long long ocs,
                                                double sign, Grid g, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const FsBin q = fs_bin(b, g);
    const double t[3] = {freq(q.kx, g.n1, g.L1, true), freq(q.ky, g.n2, g.L2, true),
                         freq(q.kz, g.n3, g.L3, true)};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
      double dx = 0.0, dy = 0.0;
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        const cplx<R> v = s[(3 * i + j) * scs + b];
        dx += t[j] * (double)v.x;
        dy += t[j] * (double)v.y;
      }
      out[i * ocs + b] = cplx<R>{(R)(-sign * dy), (R)(sign * dx)};
    }
  }
}

// z = [xi~ . Kbar . xi~]^-1 r (eq. precf with the 81-entry mean tangent, zero where
// xi~ = 0), after the Hermitian projection of r on the self-conjugate x-planes.
template <typename R>
__global__ void __launch_bounds__(256) k_fs_precond(const cplx<R>* __restrict__ r,
                                                    cplx<R>* __restrict__ z, long long cs,
                                                    const double* __restrict__ kbar81, Grid g,
                                                    const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  __shared__ double K[81];
  if (threadIdx.x < 81) K[threadIdx.x] = kbar81[threadIdx.x];
  __syncthreads();
  for (long long b = blockIdx.x * (long long)blockDim.x + threadIdx.x; b < g.nspec;
       b += (long long)gridDim.x * blockDim.x) {
    const FsBin q = fs_bin(b, g);
    const double t[3] = {freq(q.kx, g.n1, g.L1, true), freq(q.ky, g.n2, g.L2, true),
                         freq(q.kz, g.n3, g.L3, true)};
    cplx<R> ri[3] = {r[b], r[cs + b], r[2 * cs + b]};
    if (q.kx == 0 || (g.n1 % 2 == 0 && q.kx == g.n1 / 2)) {
      const int ky = (g.n2 - q.ky) % g.n2, kz = (g.n3 - q.kz) % g.n3;
      const long long bp = (long long)q.kx + (long long)g.n1h * (ky + (long long)g.n2 * kz);
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        const cplx<R> o = r[c * cs + bp];
        ri[c] = cplx<R>{R(0.5) * (ri[c].x + o.x), R(0.5) * (ri[c].y - o.y)};
      }
    }
    cplx<R> zo[3] = {{0, 0}, {0, 0}, {0, 0}};
    if (t[0] != 0.0 || t[1] != 0.0 || t[2] != 0.0) {
      double Am[9], Ai[9];
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          double s = 0.0;
#pragma unroll
          for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int l = 0; l < 3; ++l) s += t[j] * K[9 * (3 * i + j) + 3 * k + l] * t[l];
          Am[3 * i + k] = s;
        }
      if (inv3(Am, Ai)) {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
          double x = 0.0, y = 0.0;
#pragma unroll
          for (int k = 0; k < 3; ++k) {
            x += Ai[3 * i + k] * (double)ri[k].x;
            y += Ai[3 * i + k] * (double)ri[k].y;
          }
          zo[i] = cplx<R>{(R)x, (R)y};
        }
      }
    }
    z[b] = zo[0];
    z[cs + b] = zo[1];
    z[2 * cs + b] = zo[2];
  }
}

// x <- gK : x per voxel (9 real components in place)
__global__ void __launch_bounds__(256) k_fs_tangent(double* __restrict__ x, long long N,
                                                    const double* __restrict__ gK,
                                                    const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    double in[9];
#pragma unroll
    for (int c = 0; c < 9; ++c) in[c] = x[c * N + v];
#pragma unroll
    for (int r = 0; r < 9; ++r) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < 9; ++c) s += gK[(long long)(9 * r + c) * N + v] * in[c];
      x[r * N + v] = s;
    }
  }
}

// partial[c * gridDim.x + blk]: block sums of component c (blockIdx.y) of a field
__global__ void __launch_bounds__(256) k_colsum(const double* __restrict__ x, long long N,
                                                double* __restrict__ partial) {
  __shared__ double red[4];
  const int c = blockIdx.y;
  double s = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
    s += x[c * N + v];
  block_partial_sum(s, partial + (long long)c * gridDim.x, red);
}

// ---- voxel kernels of the increment ------------------------------------------------------
__global__ void __launch_bounds__(256) k_fs_add_uniform(long long N, double* __restrict__ F,
                                                        Nine9 d) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 9; ++c) F[c * N + v] += d.v[c];
}

// F += t dF; partial maxima of |t dF| and |F - F_t|
__global__ void __launch_bounds__(256) k_fs_update(long long N, double* __restrict__ F,
                                                   const double* __restrict__ dF, double t,
                                                   const double* __restrict__ Ft,
                                                   double* __restrict__ partial) {
  double mx[2] = {0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const double s = t * dF[c * N + v];
      const double f = F[c * N + v] + s;
      F[c * N + v] = f;
      mx[0] = fmax(mx[0], fabs(s));
      mx[1] = fmax(mx[1], fabs(f - Ft[c * N + v]));
    }
  block_partials<2, true>(mx, partial);
}

// maxima |F - F_prev|, |F - F_t|, |phi - phi_prev|, |phi - phi_t|
__global__ void __launch_bounds__(256) k_fs_stag_norms(long long N, const double* __restrict__ F,
                                                       const double* __restrict__ Fprev,
                                                       const double* __restrict__ Ft,
                                                       const double* __restrict__ phi,
                                                       const double* __restrict__ phi_prev,
                                                       const double* __restrict__ phi_t,
                                                       double* __restrict__ partial) {
  double mx[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      const double f = F[c * N + v];
      mx[0] = fmax(mx[0], fabs(f - Fprev[c * N + v]));
      mx[1] = fmax(mx[1], fabs(f - Ft[c * N + v]));
    }
    mx[2] = fmax(mx[2], fabs(phi[v] - phi_prev[v]));
    mx[3] = fmax(mx[3], fabs(phi[v] - phi_t[v]));
  }
  block_partials<4, true>(mx, partial);
}

// Driving state S = (l / Gc) <W_e+ + W_p + dW_p - W_crit> once triggered (eq. zeta), and the
// partial sums of S and S^2.
__global__ void __launch_bounds__(256) k_fs_source(long long N, const double* __restrict__ aux,
                                                   const double* __restrict__ wp,
                                                   const double* __restrict__ trig,
                                                   const double* __restrict__ wcrit,
                                                   double* __restrict__ S, Material m,
                                                   double* __restrict__ partial) {
  double acc[2] = {0.0, 0.0};
  const double c = m.ell / m.Gc;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
    if (trig[v] != 0.0) s = c * fmax(0.0, aux[3 * N + v] + wp[v] + aux[v] - wcrit[v]);
    S[v] = s;
    acc[0] += s;
    acc[1] += s * s;
  }
  block_partials<2, false>(acc, partial);
}

// History commit (FP64): Fp, strength (linear hardening), SSD density, plastic work,
// stored energy density, tensile-energy history, trigger and threshold (eq. crit).
// Partials: 9 sums of g(phi) P, 9 sums of F, the number of triggered voxels (19 sums at
// partial[0 .. 19 nb)), then the maxima of phi and of phi over the voxels that can slip
// (2 at partial[19 nb ..)).
__global__ void __launch_bounds__(256)
k_fs_commit(long long N, const double* __restrict__ P, const double* __restrict__ F,
            double* __restrict__ Fp, const double* __restrict__ fp_tr, double* __restrict__ gslip,
            double* __restrict__ rho_ssd, const double* __restrict__ rho_gnd,
            double* __restrict__ wp, double* __restrict__ gs, double* __restrict__ H,
            double* __restrict__ wcrit, double* __restrict__ trig, const double* __restrict__ aux,
            const double* __restrict__ phi, Material m, double* __restrict__ partial) {
  double sums[19];
  double mx[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 19; ++c) sums[c] = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 9; ++c) Fp[c * N + v] = fp_tr[c * N + v];
    const double g0 = gslip[v];
    const bool slips = isfinite(g0);
    if (m.flow == FLOW_POWER && slips) gslip[v] = g0 + m.h_lin * aux[N + v];
    const double rs = rho_ssd[v] + m.lambda_ssd * sqrt(2.0 / 3.0 * aux[2 * N + v]);
    rho_ssd[v] = rs;
    const double dw = aux[v];
    const double w = wp[v] + dw;
    wp[v] = w;
    const double G = gs[v] + m.xi_store * dw / sqrt(rs + rho_gnd[v]);
    gs[v] = G;
    const double h = fmax(H[v], aux[3 * N + v]);
    H[v] = h;
    double tr = trig[v];
    if (tr == 0.0 && G >= m.G_crit) {
      wcrit[v] = h + w;
      tr = 1.0;
      trig[v] = 1.0;
    }
    const double ph = phi[v];
    const double gphi = (1.0 - ph) * (1.0 - ph) + m.kres;
#pragma unroll
    for (int c = 0; c < 9; ++c) {
      sums[c] += gphi * P[c * N + v];
      sums[9 + c] += F[c * N + v];
    }
    sums[18] += tr;
    mx[0] = fmax(mx[0], ph);
    if (slips) mx[1] = fmax(mx[1], ph);
  }
  block_partials<19, false>(sums, partial);
  block_partials<2, true>(mx, partial + 19LL * gridDim.x);
}

// out = g(phi) P (9 components)
__global__ void __launch_bounds__(256) k_fs_degrade(long long N, const double* __restrict__ P,
                                                    const double* __restrict__ phi, double kres,
                                                    double* __restrict__ out) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double gphi = (1.0 - phi[v]) * (1.0 - phi[v]) + kres;
#pragma unroll
    for (int c = 0; c < 9; ++c) out[c * N + v] = gphi * P[c * N + v];
  }
}

int fs_grid(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

}  // namespace

// ---- launchers ------------------------------------------------------------------------------
void launch_fs_constitutive(long long N, const double* F, const double* dF, double t,
                            const double* Fpn, const double* gslip, const int* grain,
                            const double* gtab, double* Sws, const double* phi, double* P,
                            double* fp_tr, double* aux, double* gK, const FsFrame& fr,
                            const Material& m, int* fail, hipStream_t st) {
  const int nb = (int)((N + 63) / 64);
  if (m.flow == FLOW_DUNNE)
    hipLaunchKernelGGL((k_fs_constitutive<FLOW_DUNNE>), dim3(nb), dim3(64), 0, st, N, F, dF, t, Fpn,
                       gslip, grain, gtab, Sws, phi, P, fp_tr, aux, gK, fr, m, fail);
  else
    hipLaunchKernelGGL((k_fs_constitutive<FLOW_POWER>), dim3(nb), dim3(64), 0, st, N, F, dF, t, Fpn,
                       gslip, grain, gtab, Sws, phi, P, fp_tr, aux, gK, fr, m, fail);
}

void launch_fs_grad(const Plans& p, const cplx<double>* u, long long ucs, cplx<double>* e,
                    long long ecs, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_fs_grad<double>), dim3(fs_grid(p.g.nspec)), dim3(256), 0, st, u, ucs, e,
                     ecs, p.g, stop);
}

void launch_fs_div(const Plans& p, const cplx<double>* s, long long scs, cplx<double>* out,
                   long long ocs, double sign, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_fs_div<double>), dim3(fs_grid(p.g.nspec)), dim3(256), 0, st, s, scs, out,
                     ocs, sign, p.g, stop);
}

void launch_fs_precond(const Plans& p, const cplx<double>* r, cplx<double>* z, long long cs,
                       const double* kbar81, hipStream_t st, const double* stop) {
  hipLaunchKernelGGL((k_fs_precond<double>), dim3(fs_grid(p.g.nspec)), dim3(256), 0, st, r, z, cs,
                     kbar81, p.g, stop);
}

void launch_fs_tangent(double* x, long long N, const double* gK, hipStream_t st,
                       const double* stop) {
  hipLaunchKernelGGL(k_fs_tangent, dim3(fs_grid(N)), dim3(256), 0, st, x, N, gK, stop);
}

int launch_colsum(const double* x, long long N, int ncomp, double* partial, hipStream_t st) {
  long long b = (N + 255) / 256;
  const int nb = (int)(b < 256 ? (b < 1 ? 1 : b) : 256);
  hipLaunchKernelGGL(k_colsum, dim3(nb, ncomp), dim3(256), 0, st, x, N, partial);
  return nb;
}

void launch_fs_add_uniform(long long N, double* F, const double d[9], hipStream_t st) {
  Nine9 dd;
  for (int c = 0; c < 9; ++c) dd.v[c] = d[c];
  hipLaunchKernelGGL(k_fs_add_uniform, dim3(fs_grid(N)), dim3(256), 0, st, N, F, dd);
}

void launch_fs_update(long long N, double* F, const double* dF, double t, const double* Ft,
                      double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_fs_update, dim3(voxel_grid(N)), dim3(256), 0, st, N, F, dF, t, Ft, partial);
}

void launch_fs_stag_norms(long long N, const double* F, const double* Fprev, const double* Ft,
                          const double* phi, const double* phi_prev, const double* phi_t,
                          double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_fs_stag_norms, dim3(voxel_grid(N)), dim3(256), 0, st, N, F, Fprev, Ft, phi,
                     phi_prev, phi_t, partial);
}

void launch_fs_source(long long N, const double* aux, const double* wp, const double* trig,
                      const double* wcrit, double* S, const Material& m, double* partial,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_fs_source, dim3(voxel_grid(N)), dim3(256), 0, st, N, aux, wp, trig, wcrit,
                     S, m, partial);
}

void launch_fs_commit(long long N, const double* P, const double* F, double* Fp,
                      const double* fp_tr, double* gslip, double* rho_ssd, const double* rho_gnd,
                      double* wp, double* gs, double* H, double* wcrit, double* trig,
                      const double* aux, const double* phi, const Material& m, double* partial,
                      hipStream_t st) {
  hipLaunchKernelGGL(k_fs_commit, dim3(voxel_grid(N)), dim3(256), 0, st, N, P, F, Fp, fp_tr, gslip,
                     rho_ssd, rho_gnd, wp, gs, H, wcrit, trig, aux, phi, m, partial);
}

void launch_fs_degrade(long long N, const double* P, const double* phi, double kres, double* out,
                       hipStream_t st) {
  hipLaunchKernelGGL(k_fs_degrade, dim3(fs_grid(N)), dim3(256), 0, st, N, P, phi, kres, out);
}

}  // namespace rvefft
