// Per-voxel kernels: crystal-plasticity update with consistent tangent, the
// phase-field driving state, the history commit and the GND density (Sec. 2).
//
// Constitutive model (small-strain form of Sec. 2.1): tau_a = P_a : sigma with
// P_a = sym(s_a (x) n_a), and one of two flow rules for the slip increment,
//   power law:             dgamma_a = dt gdot0 sign(tau_a) |tau_a / g|^n,
//   thermally activated:   dgamma_a = dt A sign(tau_a) sinh(beta <|tau_a| - g>)
//                          (eq. flowrule, A = rho_m b^2 v_D exp(-dF/kT), beta = dV/kT);
// backward Euler on sigma with g frozen over the step:
//   R(sigma) = C^-1 (sigma - sigma_tr) + sum_a dgamma_a P_a = 0,
//   sigma_tr = C (eps - eps_p).
// R is the gradient of a strictly convex potential Phi; the root is found by a
// Newton iteration with backtracking on Phi (FP64 in every precision mode), and
// the consistent tangent is K = (C^-1 + sum_a d dgamma_a / d tau_a P_a P_a^T)^-1.
// All 6x6 algebra is in the Mandel basis.
#include "cpdev.h"

namespace rvefft {

int voxel_grid(long long n) {
  long long b = (n + 255) / 256;
  return (int)(b < 2048 ? (b < 1 ? 1 : b) : 2048);
}

// Slip increments at stress sig (Mandel) with the flow rule of m: tau and dgamma.
__device__ __forceinline__ void slip(const double* __restrict__ P, const double sig[6], double g,
                                     const Material& m, double tau[12], double dg[12]) {
  const Flow f = make_flow(m, g);
#pragma unroll
  for (int a = 0; a < 12; ++a) {
    double s = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) s += P[a * 6 + b] * sig[b];
    tau[a] = s;
    double d, dd;
    if (m.flow == FLOW_DUNNE) slip_law<FLOW_DUNNE>(f, s, d, dd);
    else slip_law<FLOW_POWER>(f, s, d, dd);
    dg[a] = d;
  }
}

// The return map runs in the crystal frame: there the Schmid tensors and the cubic
// stiffness are the same for every grain (kernel-argument constants, read through the
// scalar unit), so only the stress state of a voxel occupies vector registers.  The
// potential, residual and tangent are invariant under the (orthogonal) Mandel rotation.

// Phi(sig) = 1/2 (sig-sig_tr) S (sig-sig_tr) + sum of the systems' potential shares
template <int F>
__device__ __forceinline__ double potential(const CrystalFrame& cf, const double sig[6],
                                            const double str[6], const Flow& f) {
  double d[6], Sd[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) d[i] = sig[i] - str[i];
  cubic_mul(cf.s11, cf.s12, cf.s66, d, Sd);
  double el = 0.0;
#pragma unroll
  for (int i = 0; i < 6; ++i) el += d[i] * Sd[i];
  double pl = 0.0;
#pragma unroll 1
  for (int a = 0; a < 12; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) t += cf.P[a * 6 + b] * sig[b];
    pl += slip_pot<F>(f, t);
  }
  return 0.5 * el + pot_scale<F>(f) * pl;
}

// Residual R = S (sig - sig_tr) + sum dgamma P and packed Jacobian J (21), accumulated
// slip system by slip system; with phi, also Phi(sig) (the power law's from the same
// resolved stresses and powers, the same arithmetic as potential()).
template <int F>
__device__ __forceinline__ void resjac(const CrystalFrame& cf, const double sig[6],
                                       const double str[6], const Flow& f, double Rv[6],
                                       double J[21], double* phi = nullptr) {
  double d[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) d[i] = sig[i] - str[i];
  cubic_mul(cf.s11, cf.s12, cf.s66, d, Rv);
  constexpr bool POW = F == FLOW_POWER;
  double el = 0.0, pl = 0.0;
  if (POW && phi) {
#pragma unroll
    for (int i = 0; i < 6; ++i) el += d[i] * Rv[i];
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j)
      J[pk(i, j)] = (i == j) ? (i < 3 ? cf.s11 : cf.s66) : ((j < 3) ? cf.s12 : 0.0);
#pragma unroll 1
  for (int a = 0; a < 12; ++a) {
    double t = 0.0;
#pragma unroll
    for (int b = 0; b < 6; ++b) t += cf.P[a * 6 + b] * sig[b];
    double dg, ddg;
    if constexpr (POW) {
      double pot;
      slip_law_pot_power(f, t, dg, ddg, pot);
      if (phi) pl += pot;
    } else {
      slip_law<F>(f, t, dg, ddg);
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      Rv[i] += dg * cf.P[a * 6 + i];
      const double di = ddg * cf.P[a * 6 + i];
#pragma unroll
      for (int j = i; j < 6; ++j) J[pk(i, j)] += di * cf.P[a * 6 + j];
    }
  }
  if (phi) *phi = POW ? 0.5 * el + pot_scale<F>(f) * pl : potential<F>(cf, sig, str, f);
}

// Solve the return map with Newton steps and a backtracking line search on Phi.  sig
// (crystal-frame Mandel, in/out) holds a warm start.  With the thermally activated rule
// the iteration starts from it or from the trial stress scaled into the elastic range,
// whichever has the lower potential (far above the threshold of the exponential rule the
// Newton steps shrink to the rule's stress scale 1/beta, or the potential overflows);
// the power law starts from the warm start.  The root does not depend on the start.
// Returns the number of Newton iterations, or -1 if it did not converge.
template <int F>
__device__ int return_map(const CrystalFrame& cf, const double str[6], const Flow& f,
                          double sig[6]) {
  if constexpr (F == FLOW_DUNNE) {
    double tmax = 0.0;
#pragma unroll 1
    for (int a = 0; a < 12; ++a) {
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < 6; ++b) t += cf.P[a * 6 + b] * str[b];
      tmax = fmax(tmax, fabs(t));
    }
    const double sc = fmin(1.0, 1.0 / fmax(tmax * f.ig, 1e-300));
    double sd[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) sd[i] = sc * str[i];
    const double pw = potential<F>(cf, sig, str, f);
    const double pd = potential<F>(cf, sd, str, f);
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
    double Rv[6], J[21], d[6], mR[6], phi0;
    resjac<F>(cf, sig, str, f, Rv, J, &phi0);
    if (!chol6p(J)) return -1;
#pragma unroll
    for (int i = 0; i < 6; ++i) mR[i] = -Rv[i];
    chol6p_solve(J, mR, d);
    double slope = 0.0;
#pragma unroll
    for (int i = 0; i < 6; ++i) slope += Rv[i] * d[i];
    double t = 1.0;
    for (int ls = 0; ls < 60; ++ls) {
      double c[6];
#pragma unroll
      for (int i = 0; i < 6; ++i) c[i] = sig[i] + t * d[i];
      const double phi1 = potential<F>(cf, c, str, f);   // inf past an overflow: halve
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
  // one polishing Newton step at the root
  {
    double Rv[6], J[21], d[6];
    resjac<F>(cf, sig, str, f, Rv, J);
    if (!chol6p(J)) return -1;
    chol6p_solve(J, Rv, d);
#pragma unroll
    for (int i = 0; i < 6; ++i) sig[i] -= d[i];
  }
  return it + 1;
}

__device__ __forceinline__ void load6(const double* __restrict__ f, long long N, long long v, double o[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) o[c] = f[c * N + v];
}

// Component c of a component-major field at byte offset boff (< 4 GiB): the component
// base is uniform (scalar registers) and the lane offset 32 bits, so a voxel's many
// component accesses share one offset register instead of a 64-bit address each.
template <typename T>
__device__ __forceinline__ T& comp(T* f, long long N, int c, unsigned boff) {
  return *(T*)((char*)(f + c * N) + boff);
}
template <typename T>
__device__ __forceinline__ const T& comp(const T* f, long long N, int c, unsigned boff) {
  return *(const T*)((const char*)(f + c * N) + boff);
}
__device__ __forceinline__ void load6o(const double* __restrict__ f, long long N, unsigned boff,
                                       double o[6]) {
#pragma unroll
  for (int c = 0; c < 6; ++c) o[c] = comp(f, N, c, boff);
}

// ---------------------------------------------------------------------------
// Constitutive update at eps + t*deps.  Writes sigma (tensor comps), g(phi) K (21
// Mandel entries) and g(phi) w per voxel, with w = 1/2 sig_tr S sig_tr - Phi(sig) the
// incremental energy.
// Symmetric-tensor rotations with the grain rotation Rm (crystal -> sample, row-major
// 3x3): tensor components xx, yy, zz, yz, xz, xy.
// crystal-frame components of the sample-frame tensor t: Rm^T T Rm
__device__ __forceinline__ void to_crystal(const double* Rm, const double t[6], double o[6]) {
  double T[3][3], W[3][3];
  sym33(t, T);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      W[i][l] = T[i][0] * Rm[0 * 3 + l] + T[i][1] * Rm[1 * 3 + l] + T[i][2] * Rm[2 * 3 + l];
  auto c = [&](int k, int l) {
    return Rm[0 * 3 + k] * W[0][l] + Rm[1 * 3 + k] * W[1][l] + Rm[2 * 3 + k] * W[2][l];
  };
  o[0] = c(0, 0); o[1] = c(1, 1); o[2] = c(2, 2); o[3] = c(1, 2); o[4] = c(0, 2); o[5] = c(0, 1);
}
// sample-frame components of the crystal-frame tensor t: Rm T Rm^T
__device__ __forceinline__ void to_sample(const double* Rm, const double t[6], double o[6]) {
  double T[3][3], W[3][3];
  sym33(t, T);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int l = 0; l < 3; ++l)
      W[i][l] = T[i][0] * Rm[l * 3 + 0] + T[i][1] * Rm[l * 3 + 1] + T[i][2] * Rm[l * 3 + 2];
  auto c = [&](int k, int l) {
    return Rm[k * 3 + 0] * W[0][l] + Rm[k * 3 + 1] * W[1][l] + Rm[k * 3 + 2] * W[2][l];
  };
  o[0] = c(0, 0); o[1] = c(1, 1); o[2] = c(2, 2); o[3] = c(1, 2); o[4] = c(0, 2); o[5] = c(0, 1);
}

// Three waves per SIMD (at most 168 VGPRs): the extra occupancy hides more of the FP64
// latencies than the spills it causes cost (measured 15 % faster than the unconstrained
// two waves; a four-wave bound spills far more and runs at half speed).
template <typename R, int F>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3, 8)))
k_constitutive(long long N, const double* __restrict__ eps, const double* __restrict__ deps,
               double t, const double* __restrict__ epsp, const double* __restrict__ gslip,
               const int* __restrict__ grain, const double* __restrict__ gtab,
               double* __restrict__ sig_io, const double* __restrict__ phi, R* __restrict__ gK,
               double* __restrict__ gw, CrystalFrame cf, Material m, int* __restrict__ fail,
               double* __restrict__ sums) {
  // one voxel per thread (N < 2^29, so byte offsets fit 32 bits)
  const unsigned v = blockIdx.x * blockDim.x + threadIdx.x;
  // with sums: the block partials of the constitutive sums (sum gK as stored, sum g w,
  // sum g(phi) sigma; the layout of k_const_sums), formed from the values as they are
  // written instead of a second pass over the fields
  double acc[RED_CONST];
  if (v < N) {
    const unsigned b8 = v * 8u, bR = v * (unsigned)sizeof(R);
    // grain rotation crystal -> sample: read before the return map and again after it
    // (the second read through an offset the compiler cannot see through, so that the
    // nine values are not held in registers across the Newton iteration)
    const double* gR = gtab + (long long)comp(grain, N, 0, v * 4u) * GT_STRIDE + GT_R;
    double e[6], ep[6], s0[6], de[6], ec[6], str[6], sig[6];
    load6o(eps, N, b8, e);
    if (deps) {
      load6o(deps, N, b8, de);
#pragma unroll
      for (int c = 0; c < 6; ++c) e[c] += t * de[c];
    }
    load6o(epsp, N, b8, ep);
    load6o(sig_io, N, b8, s0);
#pragma unroll
    for (int c = 0; c < 6; ++c) e[c] -= ep[c];
    {
      double Rm0[9], tc[6];
#pragma unroll
      for (int i = 0; i < 9; ++i) Rm0[i] = gR[i];
      to_crystal(Rm0, e, tc);
      to_mandel(tc, ec);
      to_crystal(Rm0, s0, tc);
      to_mandel(tc, sig);
    }
    cubic_mul(cf.c11, cf.c12, cf.c66, ec, str);
    const Flow f = make_flow(m, comp(gslip, N, 0, b8));
    const int its = return_map<F>(cf, str, f, sig);
    if (its < 0) atomicAdd(fail, 1);
    double Rm[9];
    {
      int roff = 0;
      asm volatile("" : "+v"(roff));
#pragma unroll
      for (int i = 0; i < 9; ++i) Rm[i] = gR[i + roff];
    }
    // tangent at the root, crystal frame
    double Rv[6], J[21], phi_root;
    resjac<F>(cf, sig, str, f, Rv, J, &phi_root);
    double K[21];
    if (chol6p(J)) chol6p_inverse(J, K);
    else {
      atomicAdd(fail, 1);
#pragma unroll
      for (int c = 0; c < 21; ++c) K[c] = 0.0;
    }
    const double q = 1.0 - comp(phi, N, 0, b8);
    const double gphi = q * q + m.kres;
    // incremental energy (frame invariant)
    {
      double Ss[6];
      cubic_mul(cf.s11, cf.s12, cf.s66, str, Ss);
      double el = 0.0;
#pragma unroll
      for (int i = 0; i < 6; ++i) el += str[i] * Ss[i];
      const double wv = gphi * (0.5 * el - phi_root);
      comp(gw, N, 0, b8) = wv;
      acc[21] = wv;
    }
    // back to the sample frame: sigma = Rm sig Rm^T; gK = g(phi) Q K Q^T with Q the
    // Mandel form of the rotation, Q_IJ = (w_I / w_J) (R_ik R_jl + [k != l] R_il R_jk)
    // for the index pairs I = (i, j), J = (k, l) and Mandel weights w (1 or sqrt 2)
    {
      double tc[6], st[6];
      from_mandel(sig, tc);
      to_sample(Rm, tc, st);
#pragma unroll
      for (int c = 0; c < 6; ++c) {
        comp(sig_io, N, c, b8) = st[c];
        acc[22 + c] = gphi * st[c];
      }
    }
    double Q[36];
    {
      constexpr int pi[6] = {0, 1, 2, 1, 0, 0}, pj[6] = {0, 1, 2, 2, 2, 1};
      const double s2 = 1.41421356237309504880, is2 = 0.70710678118654752440;
#pragma unroll
      for (int I = 0; I < 6; ++I)
#pragma unroll
        for (int J = 0; J < 6; ++J) {
          const int i = pi[I], j = pj[I], k = pi[J], l = pj[J];
          const double wi = (I < 3) ? 1.0 : s2;
          Q[I * 6 + J] = (J < 3) ? wi * Rm[i * 3 + k] * Rm[j * 3 + k]
                                 : wi * is2 * (Rm[i * 3 + k] * Rm[j * 3 + l] +
                                               Rm[i * 3 + l] * Rm[j * 3 + k]);
        }
    }
#pragma unroll
    for (int i = 0; i < 6; ++i) {
      double u[6];                 // row i of Q K
#pragma unroll
      for (int l = 0; l < 6; ++l) {
        double a = 0.0;
#pragma unroll
        for (int k = 0; k < 6; ++k) a += Q[i * 6 + k] * K[pk(k, l)];
        u[l] = a;
      }
#pragma unroll
      for (int j = i; j < 6; ++j) {
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < 6; ++l) a += u[l] * Q[j * 6 + l];
        const R kv = (R)(gphi * a);
        comp(gK, N, pk(i, j), bR) = kv;
        acc[pk(i, j)] = (double)kv;
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < RED_CONST; ++c) acc[c] = 0.0;
  }
  if (sums) block_partials<RED_CONST, false>(acc, sums);
}

// ---------------------------------------------------------------------------
// Pointwise plane stress of plates one voxel thick (Sec. 4.1-4.3): the out-of-plane
// stress (Mandel O = zz, yz, xz = 2, 3, 4) vanishes at every voxel and the out-of-plane
// strain is a local unknown.  Each Newton step eliminates it by static condensation of
// the linearised point:
//   d e_O = -B d e_P - r,   B = K_OO^-1 K_OP,   r = K_OO^-1 sigma_O,
// so that the in-plane balance sees the tangent K_PP - K_PO B (the stiffness of the
// constrained point) and the stress sigma_P - B^T sigma_O (P = xx, yy, xy = 0, 1, 5).
// This pass rewrites gK in place: the PP block condensed, the PO block zero and the OO
// block kept (so the displacement u_z, whose equation then decouples with a zero right
// side, stays zero in the Krylov solve); it writes the condensed effective stress (tensor
// components, out-of-plane ones zero) and, per voxel, B (9, row-major over O x P) and r
// (3, Mandel, undegraded) for the recovery of d e_O.
template <typename R>
__global__ void __launch_bounds__(256)
k_plane_condense(long long N, R* __restrict__ gK, const double* __restrict__ sig,
                 const double* __restrict__ phi, double kres, double* __restrict__ sig_c,
                 double* __restrict__ rec, int* __restrict__ fail) {
  constexpr int Pi[3] = {0, 1, 5}, Oi[3] = {2, 3, 4};
  const double s2 = 1.41421356237309504880, is2 = 0.70710678118654752440;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    double K[21];
#pragma unroll
    for (int c = 0; c < 21; ++c) K[c] = (double)gK[c * N + v];
    double sm[6];
#pragma unroll
    for (int c = 0; c < 6; ++c) sm[c] = (c < 3 ? 1.0 : s2) * sig[c * N + v];
    const double q = 1.0 - phi[v];
    const double gphi = q * q + kres;
    // inverse of the SPD 3x3 block K_OO by cofactors
    const double a00 = K[pk(2, 2)], a01 = K[pk(2, 3)], a02 = K[pk(2, 4)];
    const double a11 = K[pk(3, 3)], a12 = K[pk(3, 4)], a22 = K[pk(4, 4)];
    const double c00 = a11 * a22 - a12 * a12, c01 = a02 * a12 - a01 * a22,
                 c02 = a01 * a12 - a02 * a11, c11 = a00 * a22 - a02 * a02,
                 c12 = a01 * a02 - a00 * a12, c22 = a00 * a11 - a01 * a01;
    const double det = a00 * c00 + a01 * c01 + a02 * c02;
    if (!(det > 0.0) || !isfinite(det)) {
      atomicAdd(fail, 1);
      continue;
    }
    const double id = 1.0 / det;
    const double Ai[3][3] = {{c00 * id, c01 * id, c02 * id},
                             {c01 * id, c11 * id, c12 * id},
                             {c02 * id, c12 * id, c22 * id}};
    double B[3][3], r[3], so[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) so[a] = sm[Oi[a]];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = 0.0;
#pragma unroll
        for (int b = 0; b < 3; ++b) t += Ai[a][b] * K[pk(Oi[b], Pi[j])];
        B[a][j] = t;
      }
      double t = 0.0;
#pragma unroll
      for (int b = 0; b < 3; ++b) t += Ai[a][b] * so[b];
      r[a] = gphi * t;          // gK = g K: K_OO^-1 sigma_O = g (gK_OO)^-1 sigma_O
    }
    double Kc[3][3], sc[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = 0; j < 3; ++j) {
        double t = K[pk(Pi[i], Pi[j])];
#pragma unroll
        for (int a = 0; a < 3; ++a) t -= K[pk(Pi[i], Oi[a])] * B[a][j];
        Kc[i][j] = t;
      }
      double t = sm[Pi[i]];
#pragma unroll
      for (int a = 0; a < 3; ++a) t -= B[a][i] * so[a];
      sc[i] = t;
    }
#pragma unroll
    for (int i = 0; i < 3; ++i) {
#pragma unroll
      for (int j = i; j < 3; ++j) gK[pk(Pi[i], Pi[j]) * N + v] = (R)(0.5 * (Kc[i][j] + Kc[j][i]));
#pragma unroll
      for (int a = 0; a < 3; ++a) gK[pk(Pi[i], Oi[a]) * N + v] = (R)0.0;
    }
    sig_c[0 * N + v] = sc[0];
    sig_c[1 * N + v] = sc[1];
    sig_c[5 * N + v] = is2 * sc[2];
    sig_c[2 * N + v] = 0.0;
    sig_c[3 * N + v] = 0.0;
    sig_c[4 * N + v] = 0.0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
      for (int j = 0; j < 3; ++j) rec[(3 * a + j) * N + v] = B[a][j];
      rec[(9 + a) * N + v] = r[a];
    }
  }
}

// d e_O = -B d e_P - r on the Newton correction (tensor components)
__global__ void __launch_bounds__(256) k_plane_recover(long long N, double* __restrict__ deps,
                                                       const double* __restrict__ rec) {
  const double s2 = 1.41421356237309504880, is2 = 0.70710678118654752440;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double dp[3] = {deps[0 * N + v], deps[1 * N + v], s2 * deps[5 * N + v]};
    double dO[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      double t = -rec[(9 + a) * N + v];
#pragma unroll
      for (int j = 0; j < 3; ++j) t -= rec[(3 * a + j) * N + v] * dp[j];
      dO[a] = t;
    }
    deps[2 * N + v] = dO[0];
    deps[3 * N + v] = is2 * dO[1];
    deps[4 * N + v] = is2 * dO[2];
  }
}

void launch_plane_recover(long long N, double* deps, const double* rec, hipStream_t st) {
  hipLaunchKernelGGL(k_plane_recover, dim3(voxel_grid(N)), dim3(256), 0, st, N, deps, rec);
}

// Block partials of the constitutive sums: sum gK (21), sum g w, sum g(phi) sigma (6).
template <typename R>
__global__ void __launch_bounds__(256)
k_const_sums(long long N, const R* __restrict__ gK, const double* __restrict__ gw,
             const double* __restrict__ sig, const double* __restrict__ phi, double kres,
             double* __restrict__ partial) {
  double acc[RED_CONST];
#pragma unroll
  for (int c = 0; c < RED_CONST; ++c) acc[c] = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    // streamed: the tangent's next readers are the x passes (at 128^3: 132 against 153 us)
#pragma unroll
    for (int c = 0; c < 21; ++c)
      acc[c] += (double)__builtin_nontemporal_load(gK + (long long)c * N + v);
    acc[21] += gw[v];
    const double q = 1.0 - phi[v];
    const double gphi = q * q + kres;
#pragma unroll
    for (int c = 0; c < 6; ++c) acc[22 + c] += gphi * sig[c * N + v];
  }
  block_partials<RED_CONST, false>(acc, partial);
}

template <typename R>
int launch_constitutive(long long N, const double* eps, const double* deps, double t,
                        const double* epsp, const double* gslip, const int* grain,
                        const double* gtab, double* sig, const double* phi, R* gK, double* gw,
                        const CrystalFrame& cf, const Material& m, double* partial, int* fail,
                        hipStream_t st, double* ps_sig, double* ps_rec) {
  const int nb = (int)((N + 255) / 256);
  // plane stress condenses the tangent after the return map: its sums take a pass of
  // their own after the condensation
  double* fused = ps_sig ? nullptr : partial;
  if (m.flow == FLOW_DUNNE)
    hipLaunchKernelGGL((k_constitutive<R, FLOW_DUNNE>), dim3(nb < 1 ? 1 : nb), dim3(256), 0, st, N,
                       eps, deps, t, epsp, gslip, grain, gtab, sig, phi, gK, gw, cf, m, fail, fused);
  else
    hipLaunchKernelGGL((k_constitutive<R, FLOW_POWER>), dim3(nb < 1 ? 1 : nb), dim3(256), 0, st, N,
                       eps, deps, t, epsp, gslip, grain, gtab, sig, phi, gK, gw, cf, m, fail, fused);
  if (fused) return nb < 1 ? 1 : nb;
  hipLaunchKernelGGL((k_plane_condense<R>), dim3(voxel_grid(N)), dim3(256), 0, st, N, gK, sig,
                     phi, m.kres, ps_sig, ps_rec, fail);
  hipLaunchKernelGGL((k_const_sums<R>), dim3(voxel_grid(N)), dim3(256), 0, st, N, gK, gw, sig,
                     phi, m.kres, partial);
  return voxel_grid(N);
}
template int launch_constitutive<double>(long long, const double*, const double*, double,
                                          const double*, const double*, const int*, const double*,
                                          double*, const double*, double*, double*,
                                          const CrystalFrame&, const Material&, double*, int*,
                                          hipStream_t, double*, double*);
template int launch_constitutive<float>(long long, const double*, const double*, double,
                                         const double*, const double*, const int*, const double*,
                                         double*, const double*, float*, double*,
                                         const CrystalFrame&, const Material&, double*, int*,
                                         hipStream_t, double*, double*);

// ---------------------------------------------------------------------------

// 1/2 eps+ : C : eps+ with eps+ the positive spectral part of the elastic strain
// (tensor comps), C Mandel (eq. decMiehe, small-strain reading).
__device__ double tensile_energy(const double ee[6], const double* __restrict__ C) {
  double a[3][3] = {{ee[0], ee[5], ee[4]}, {ee[5], ee[1], ee[3]}, {ee[4], ee[3], ee[2]}};
  double d[3], V[3][3];
  jacobi3(a, d, V);
  double P[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += fmax(d[k], 0.0) * V[i][k] * V[j][k];
      P[i][j] = s;
    }
  const double pt[6] = {P[0][0], P[1][1], P[2][2], P[1][2], P[0][2], P[0][1]};
  double pm[6];
  to_mandel(pt, pm);
  double e = 0.0;
  for (int i = 0; i < 6; ++i) {
    double s = 0.0;
    for (int j = 0; j < 6; ++j) s += C[i * 6 + j] * pm[j];
    e += pm[i] * s;
  }
  return 0.5 * e;
}

// Driving state of the phase field (eq. zeta, read as S = (l/Gc) <W - W_crit> after
// the stored-energy threshold is reached) from the converged effective stress:
// trial slip, trial plastic work and the tensile elastic energy.
__global__ void __launch_bounds__(256) k_source(long long N, const double* __restrict__ eps, const double* __restrict__ sig,
                         const double* __restrict__ epsp, const double* __restrict__ gslip,
                         const int* __restrict__ grain, const double* __restrict__ gtab,
                         const double* __restrict__ wp, const double* __restrict__ trig,
                         const double* __restrict__ wcrit, double* __restrict__ S_out,
                         double* __restrict__ wep_out, Material m, double* __restrict__ partial) {
  double acc[RED_SOURCE] = {0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double* gt = gtab + (long long)grain[v] * GT_STRIDE;
    const double* P = gt + GT_P;
    double st[6], sm[6], e[6], ep[6];
    load6(sig, N, v, st);
    load6(eps, N, v, e);
    load6(epsp, N, v, ep);
    to_mandel(st, sm);
    double tau[12], dg[12];
    slip(P, sm, gslip[v], m, tau, dg);
    double dpm[6] = {0, 0, 0, 0, 0, 0};
    double dw = 0.0;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      dw += tau[a] * dg[a];
#pragma unroll
      for (int i = 0; i < 6; ++i) dpm[i] += dg[a] * P[a * 6 + i];
    }
    double dpt[6];
    from_mandel(dpm, dpt);
    double ee[6];
#pragma unroll
    for (int i = 0; i < 6; ++i) ee[i] = e[i] - (ep[i] + dpt[i]);
    const double we = tensile_energy(ee, gt + GT_C);
    const double W = we + wp[v] + dw;
    const double S = (trig[v] != 0.0) ? m.ell / m.Gc * fmax(0.0, W - wcrit[v]) : 0.0;
    S_out[v] = S;
    wep_out[v] = we;
    acc[0] += S;
    acc[1] += S * S;
  }
  block_partials<RED_SOURCE, false>(acc, partial);
}

void launch_source(long long N, const double* eps, const double* sig, const double* epsp,
                   const double* gslip, const int* grain, const double* gtab, const double* wp,
                   const double* trig, const double* wcrit, double* S, double* wep,
                   const Material& m, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_source, dim3(voxel_grid(N)), dim3(256), 0, st, N, eps, sig, epsp, gslip,
                     grain, gtab, wp, trig, wcrit, S, wep, m, partial);
}

// History commit of one converged increment (FP64), Sec. 2.1-2.3:
// eps_p, beta_p, g (linear hardening of the power law), rho_SSD, W_p, G_s, H = max W_e+,
// W_crit.
// Partials: sums of g(phi) sigma (6), eps (6) and the trigger flag; maxima of phi
// and of phi over voxels that can slip.
__global__ void __launch_bounds__(256) k_commit(long long N, const double* __restrict__ sig, double* __restrict__ gslip,
                         double* __restrict__ epsp, double* __restrict__ beta,
                         double* __restrict__ rho_ssd, const double* __restrict__ rho_gnd,
                         double* __restrict__ wp, double* __restrict__ gs, double* __restrict__ H,
                         double* __restrict__ wcrit, double* __restrict__ trig,
                         const double* __restrict__ wep, const double* __restrict__ phi,
                         const double* __restrict__ eps, const int* __restrict__ grain,
                         const double* __restrict__ gtab, Material m,
                         double* __restrict__ partial) {
  double acc[13];
  double mx[2] = {0.0, 0.0};
#pragma unroll
  for (int c = 0; c < 13; ++c) acc[c] = 0.0;
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double* gt = gtab + (long long)grain[v] * GT_STRIDE;
    const double* P = gt + GT_P;
    const double* SN = gt + GT_SN;
    double st[6], sm[6];
    load6(sig, N, v, st);
    to_mandel(st, sm);
    const double g = gslip[v];
    double tau[12], dg[12];
    slip(P, sm, g, m, tau, dg);
    double dpm[6] = {0, 0, 0, 0, 0, 0};
    double db[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    double dw = 0.0, sabs = 0.0;
#pragma unroll
    for (int a = 0; a < 12; ++a) {
      dw += tau[a] * dg[a];
      sabs += fabs(dg[a]);
#pragma unroll
      for (int i = 0; i < 6; ++i) dpm[i] += dg[a] * P[a * 6 + i];
#pragma unroll
      for (int i = 0; i < 9; ++i) db[i] += dg[a] * SN[a * 9 + i];
    }
    double dpt[6];
    from_mandel(dpm, dpt);
#pragma unroll
    for (int i = 0; i < 6; ++i) epsp[i * N + v] += dpt[i];
    double db2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      beta[i * N + v] += db[i];
      db2 += db[i] * db[i];
    }
    if (m.flow == FLOW_POWER) gslip[v] = g + m.h_lin * sabs;   // else: Taylor, after the GND
    const double rs = rho_ssd[v] + m.lambda_ssd * sqrt(2.0 / 3.0 * db2);
    rho_ssd[v] = rs;
    const double wpn = wp[v] + dw;
    wp[v] = wpn;
    const double gsn = gs[v] + m.xi_store * dw / sqrt(rs + rho_gnd[v]);
    gs[v] = gsn;
    const double hn = fmax(H[v], wep[v]);
    H[v] = hn;
    double tr = trig[v];
    if (tr == 0.0 && gsn >= m.G_crit) {
      wcrit[v] = hn + wpn;
      tr = 1.0;
      trig[v] = 1.0;
    }
    const double q = 1.0 - phi[v];
    const double gphi = q * q + m.kres;
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      acc[c] += gphi * st[c];
      acc[6 + c] += eps[c * N + v];
    }
    acc[12] += tr;
    mx[0] = fmax(mx[0], phi[v]);
    if (isfinite(g)) mx[1] = fmax(mx[1], phi[v]);
  }
  block_partials<13, false>(acc, partial);
  __syncthreads();
  block_partials<2, true>(mx, partial + 13LL * gridDim.x);
}

void launch_commit(long long N, const double* sig, double* gslip, double* epsp, double* beta,
                   double* rho_ssd, const double* rho_gnd, double* wp, double* gs, double* H,
                   double* wcrit, double* trig, const double* wep, const double* phi,
                   const double* eps, const int* grain, const double* gtab, const Material& m,
                   double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_commit, dim3(voxel_grid(N)), dim3(256), 0, st, N, sig, gslip, epsp, beta,
                     rho_ssd, rho_gnd, wp, gs, H, wcrit, trig, wep, phi, eps, grain, gtab, m,
                     partial);
}

// GND-coupled hardening (option): the end-of-increment plastic distortion beta + d beta
// (into beta_tr, 9 components) and SSD density of the slip at the converged stress and the
// current strength, as the commit would form them.
__global__ void __launch_bounds__(256) k_trial_hardening(
    long long N, const double* __restrict__ sig, const double* __restrict__ gslip,
    const double* __restrict__ beta, const double* __restrict__ rho_ssd,
    const int* __restrict__ grain, const double* __restrict__ gtab, Material m,
    double* __restrict__ beta_tr, double* __restrict__ rho_ssd_tr) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double* gt = gtab + (long long)grain[v] * GT_STRIDE;
    double st[6], sm[6];
    load6(sig, N, v, st);
    to_mandel(st, sm);
    double tau[12], dg[12];
    slip(gt + GT_P, sm, gslip[v], m, tau, dg);
    double db2 = 0.0;
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      double d = 0.0;
#pragma unroll
      for (int a = 0; a < 12; ++a) d += dg[a] * gt[GT_SN + a * 9 + i];
      beta_tr[i * N + v] = beta[i * N + v] + d;
      db2 += d * d;
    }
    rho_ssd_tr[v] = rho_ssd[v] + m.lambda_ssd * sqrt(2.0 / 3.0 * db2);
  }
}

// The Taylor strength of the end-of-increment densities, g_next = tau_c0 + mu b sqrt(
// rho_SSD + rho_GND) (voxels that cannot slip keep g = inf), and the partial maxima of
// |g_next - g| and |g_next - g_n| over the voxels that can slip.
__global__ void __launch_bounds__(256) k_taylor_next(
    long long N, const double* __restrict__ gslip, const double* __restrict__ g_n,
    const double* __restrict__ rho_ssd_tr, const double* __restrict__ rho_gnd_tr,
    const int* __restrict__ grain, const double* __restrict__ gtab, double mu_b,
    double* __restrict__ g_next, double* __restrict__ partial) {
  double mx[2] = {0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double g = gslip[v];
    if (!isfinite(g)) {
      g_next[v] = g;
      continue;
    }
    const double tau0 = gtab[(long long)grain[v] * GT_STRIDE + GT_TAU0];
    const double gn = tau0 + mu_b * sqrt(rho_ssd_tr[v] + rho_gnd_tr[v]);
    g_next[v] = gn;
    mx[0] = fmax(mx[0], fabs(gn - g));
    mx[1] = fmax(mx[1], fabs(gn - g_n[v]));
  }
  block_partials<2, true>(mx, partial);
}

void launch_trial_hardening(long long N, const double* sig, const double* gslip,
                            const double* beta, const double* rho_ssd, const int* grain,
                            const double* gtab, const Material& m, double* beta_tr,
                            double* rho_ssd_tr, hipStream_t st) {
  hipLaunchKernelGGL(k_trial_hardening, dim3(voxel_grid(N)), dim3(256), 0, st, N, sig, gslip, beta,
                     rho_ssd, grain, gtab, m, beta_tr, rho_ssd_tr);
}

void launch_taylor_next(long long N, const double* gslip, const double* g_n,
                        const double* rho_ssd_tr, const double* rho_gnd_tr, const int* grain,
                        const double* gtab, double mu_b, double* g_next, double* partial,
                        hipStream_t st) {
  hipLaunchKernelGGL(k_taylor_next, dim3(voxel_grid(N)), dim3(256), 0, st, N, gslip, g_n,
                     rho_ssd_tr, rho_gnd_tr, grain, gtab, mu_b, g_next, partial);
}

// Aitken relaxation of the coupled strength (see launch_aitken_dots in kernels.h).
__global__ void __launch_bounds__(256) k_aitken_dots(
    long long N, const double* __restrict__ gslip, const double* __restrict__ g_next,
    const double* __restrict__ r_prev, int first, double* __restrict__ partial) {
  double s[2] = {0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double g = gslip[v];
    if (!isfinite(g)) continue;
    const double r = g_next[v] - g;
    const double rp = first ? 0.0 : r_prev[v];
    const double dr = r - rp;
    s[0] += rp * dr;
    s[1] += dr * dr;
  }
  block_partials<2, false>(s, partial);
}

__global__ void __launch_bounds__(256) k_aitken_relax(
    long long N, double* __restrict__ gslip, const double* __restrict__ g_next,
    double* __restrict__ r_prev, double omega) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double g = gslip[v];
    if (!isfinite(g)) {
      r_prev[v] = 0.0;
      continue;
    }
    const double r = g_next[v] - g;
    gslip[v] = g + omega * r;
    r_prev[v] = r;
  }
}

void launch_aitken_dots(long long N, const double* gslip, const double* g_next,
                        const double* r_prev, int first, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_aitken_dots, dim3(voxel_grid(N)), dim3(256), 0, st, N, gslip, g_next,
                     r_prev, first, partial);
}
void launch_aitken_relax(long long N, double* gslip, const double* g_next, double* r_prev,
                         double omega, hipStream_t st) {
  hipLaunchKernelGGL(k_aitken_relax, dim3(voxel_grid(N)), dim3(256), 0, st, N, gslip, g_next,
                     r_prev, omega);
}

// Taylor hardening (Sec. 2.1): g = tau_c0 + mu b sqrt(rho_SSD + rho_GND) from the
// committed densities; voxels that cannot slip (g = inf) keep their strength.
__global__ void __launch_bounds__(256) k_taylor(long long N, double* __restrict__ gslip,
                         const double* __restrict__ rho_ssd, const double* __restrict__ rho_gnd,
                         const int* __restrict__ grain, const double* __restrict__ gtab,
                         double mu_b) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    if (!isfinite(gslip[v])) continue;
    const double tau0 = gtab[(long long)grain[v] * GT_STRIDE + GT_TAU0];
    gslip[v] = tau0 + mu_b * sqrt(rho_ssd[v] + rho_gnd[v]);
  }
}

void launch_taylor(long long N, double* gslip, const double* rho_ssd, const double* rho_gnd,
                   const int* grain, const double* gtab, double mu_b, hipStream_t st) {
  hipLaunchKernelGGL(k_taylor, dim3(voxel_grid(N)), dim3(256), 0, st, N, gslip, rho_ssd, rho_gnd,
                     grain, gtab, mu_b);
}

// rho_GND = sqrt(vec(Lc)^T Q vec(Lc)) / b with Lc = R^T Lambda R (crystal frame) and
// Q = (A A^T)^-1, the squared norm of the minimum-norm split into 12 edge and 6
// screw densities (eq. nye1 and the L2-norm scheme).
__global__ void __launch_bounds__(256) k_gnd(long long N, const double* __restrict__ lam9, const int* __restrict__ grain,
                      const double* __restrict__ gtab, const double* __restrict__ Q81,
                      double burgers, double* __restrict__ rho) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double* Rm = gtab + (long long)grain[v] * GT_STRIDE + GT_R;
    double L[3][3], T[3][3], Lc[9];
    for (int i = 0; i < 9; ++i) L[i / 3][i % 3] = lam9[i * N + v];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += L[i][k] * Rm[k * 3 + j];
        T[i][j] = s;                  // Lambda R
      }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += Rm[k * 3 + i] * T[k][j];
        Lc[i * 3 + j] = s;            // R^T Lambda R
      }
    double q = 0.0;
    for (int i = 0; i < 9; ++i) {
      double s = 0.0;
      for (int j = 0; j < 9; ++j) s += Q81[i * 9 + j] * Lc[j];
      q += Lc[i] * s;
    }
    rho[v] = sqrt(fmax(q, 0.0)) / burgers;
  }
}

void launch_gnd(long long N, const double* lam9, const int* grain, const double* gtab,
                const double* Q81, double burgers, double* rho_gnd, hipStream_t st) {
  hipLaunchKernelGGL(k_gnd, dim3(voxel_grid(N)), dim3(256), 0, st, N, lam9, grain, gtab, Q81,
                     burgers, rho_gnd);
}

__global__ void __launch_bounds__(256) k_eps_update(long long N, double* __restrict__ eps, const double* __restrict__ deps,
                             double t, const double* __restrict__ eps_t, double* __restrict__ partial) {
  double mx[2] = {0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double d = t * deps[c * N + v];
      const double e = eps[c * N + v] + d;
      eps[c * N + v] = e;
      mx[0] = fmax(mx[0], fabs(d));
      mx[1] = fmax(mx[1], fabs(e - eps_t[c * N + v]));
    }
  }
  block_partials<2, true>(mx, partial);
}

void launch_eps_update(long long N, double* eps, const double* deps, double t, const double* eps_t,
                       double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_eps_update, dim3(voxel_grid(N)), dim3(256), 0, st, N, eps, deps, t, eps_t,
                     partial);
}

__global__ void __launch_bounds__(256) k_slope(long long N, const double* __restrict__ sig, const double* __restrict__ deps,
                        const double* __restrict__ phi, double kres, double* __restrict__ partial) {
  double acc[1] = {0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < 6; ++c) s += (c < 3 ? 1.0 : 2.0) * sig[c * N + v] * deps[c * N + v];
    const double q = 1.0 - phi[v];
    acc[0] += (q * q + kres) * s;
  }
  block_partials<1, false>(acc, partial);
}

void launch_slope(long long N, const double* sig, const double* deps, const double* phi,
                  double kres, double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_slope, dim3(voxel_grid(N)), dim3(256), 0, st, N, sig, deps, phi, kres,
                     partial);
}

__global__ void __launch_bounds__(256) k_stag_norms(long long N, const double* __restrict__ eps,
                             const double* __restrict__ eps_prev, const double* __restrict__ eps_t,
                             const double* __restrict__ phi, const double* __restrict__ phi_prev,
                             const double* __restrict__ phi_t, double* __restrict__ partial) {
  double mx[4] = {0.0, 0.0, 0.0, 0.0};
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
#pragma unroll
    for (int c = 0; c < 6; ++c) {
      const double e = eps[c * N + v];
      mx[0] = fmax(mx[0], fabs(e - eps_prev[c * N + v]));
      mx[1] = fmax(mx[1], fabs(e - eps_t[c * N + v]));
    }
    mx[2] = fmax(mx[2], fabs(phi[v] - phi_prev[v]));
    mx[3] = fmax(mx[3], fabs(phi[v] - phi_t[v]));
  }
  block_partials<4, true>(mx, partial);
}

void launch_stag_norms(long long N, const double* eps, const double* eps_prev, const double* eps_t,
                       const double* phi, const double* phi_prev, const double* phi_t,
                       double* partial, hipStream_t st) {
  hipLaunchKernelGGL(k_stag_norms, dim3(voxel_grid(N)), dim3(256), 0, st, N, eps, eps_prev, eps_t,
                     phi, phi_prev, phi_t, partial);
}

struct Six {
  double v[6];
};

__global__ void __launch_bounds__(256) k_add_uniform(long long N, double* __restrict__ eps, Six de) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
#pragma unroll
    for (int c = 0; c < 6; ++c) eps[c * N + v] += de.v[c];
}

void launch_add_uniform(long long N, double* eps, const double de[6], hipStream_t st) {
  Six s;
  for (int c = 0; c < 6; ++c) s.v[c] = de[c];
  hipLaunchKernelGGL(k_add_uniform, dim3(voxel_grid(N)), dim3(256), 0, st, N, eps, s);
}

__global__ void __launch_bounds__(256) k_clamp(long long N, const double* __restrict__ x, const double* __restrict__ phi_t,
                        double* __restrict__ phi) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x)
    phi[v] = fmin(1.0, fmax(phi_t[v], x[v]));
}

void launch_clamp(long long N, const double* x, const double* phi_t, double* phi, hipStream_t st) {
  hipLaunchKernelGGL(k_clamp, dim3(voxel_grid(N)), dim3(256), 0, st, N, x, phi_t, phi);
}

// out = g(phi) sig on 6 components, g(phi) = (1 - phi)^2 + k_res (eq. deg)
__global__ void __launch_bounds__(256) k_degrade(long long N, const double* __restrict__ sig,
                                                 const double* __restrict__ phi, double kres,
                                                 double* __restrict__ out) {
  for (long long v = blockIdx.x * (long long)blockDim.x + threadIdx.x; v < N;
       v += (long long)gridDim.x * blockDim.x) {
    const double q = 1.0 - phi[v];
    const double gp = q * q + kres;
#pragma unroll
    for (int c = 0; c < 6; ++c) out[c * N + v] = gp * sig[c * N + v];
  }
}
void launch_degrade(long long N, const double* sig, const double* phi, double kres, double* out,
                    hipStream_t st) {
  hipLaunchKernelGGL(k_degrade, dim3(voxel_grid(N)), dim3(256), 0, st, N, sig, phi, kres, out);
}

}  // namespace rvefft
