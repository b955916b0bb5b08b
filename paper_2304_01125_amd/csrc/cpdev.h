// Per-voxel device helpers shared by the small- and finite-strain constitutive kernels:
// Mandel conversions, the two flow rules (power law and the thermally activated glide of
// eq. flowrule) with their dissipation potentials, packed 6x6 Cholesky algebra and
// deterministic block partial sums.
#pragma once
#include "kernels.h"

namespace rvefft {

static constexpr double kSqrt2 = 1.41421356237309504880;
static constexpr double kInvSqrt2 = 0.70710678118654752440;

// Deterministic block sums of NC values: shuffles within each wave, then the
// waves in index order.  Thread c < NC writes partial[c * gridDim.x + blockIdx.x].
template <int NC, bool MAX>
__device__ void block_partials(double (&v)[NC], double* partial) {
  __shared__ double red[NC][16];
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    double x = v[c];
    for (int off = 32; off > 0; off >>= 1) {
      const double y = __shfl_down(x, off, 64);
      x = MAX ? fmax(x, y) : x + y;
    }
    if (lane == 0) red[c][wid] = x;
  }
  __syncthreads();
  if (threadIdx.x < NC) {
    double s = red[threadIdx.x][0];
    for (int w = 1; w < nw; ++w) s = MAX ? fmax(s, red[threadIdx.x][w]) : s + red[threadIdx.x][w];
    partial[(long long)threadIdx.x * gridDim.x + blockIdx.x] = s;
  }
}

__device__ __forceinline__ void to_mandel(const double t[6], double m[6]) {
  m[0] = t[0]; m[1] = t[1]; m[2] = t[2];
  m[3] = kSqrt2 * t[3]; m[4] = kSqrt2 * t[4]; m[5] = kSqrt2 * t[5];
}
__device__ __forceinline__ void from_mandel(const double m[6], double t[6]) {
  t[0] = m[0]; t[1] = m[1]; t[2] = m[2];
  t[3] = kInvSqrt2 * m[3]; t[4] = kInvSqrt2 * m[4]; t[5] = kInvSqrt2 * m[5];
}

// x^e for x >= 0: binary powering when the exponent is a small integer (ei >= 0),
// the library pow otherwise.
__device__ __forceinline__ double pow_e(double x, double e, int ei) {
  if (ei >= 0) {
    double r = 1.0, b = x;
    for (int k = ei; k; k >>= 1) {
      if (k & 1) r *= b;
      b *= b;
    }
    return r;
  }
  return pow(x, e);
}

// Flow-rule constants of one voxel over one step: c0 = dt gdot0 (power law) or dt A
// (thermally activated), c1 = n or beta; g the slip resistance (critical resolved shear
// stress), ig = 1/g (0 for a voxel that cannot slip, g = inf).
struct Flow {
  double c0, c1, g, ig;
  int nm1;   // n - 1 when n is a small integer (binary powering), else -1
};

__device__ __forceinline__ Flow make_flow(const Material& m, double g) {
  Flow f;
  const bool th = m.flow == FLOW_DUNNE;
  f.c0 = m.dt * (th ? m.A : m.gdot0);
  f.c1 = th ? m.beta : m.nexp;
  f.g = g;
  f.ig = 1.0 / g;
  f.nm1 = m.nexp_int > 0 ? m.nexp_int - 1 : -1;
  return f;
}

// Slip increment dg of one system at resolved shear stress t, and d dg / d t.
template <int F>
__device__ __forceinline__ void slip_law(const Flow& f, double t, double& dg, double& ddg) {
  if constexpr (F == FLOW_POWER) {
    const double x = t * f.ig;
    const double ax = fabs(x);
    const double pw = pow_e(ax, f.c1 - 1.0, f.nm1);       // |x|^(n-1)
    dg = f.c0 * copysign(ax * pw, x);
    ddg = f.c0 * f.c1 * f.ig * pw;
  } else {
    const double o = fabs(t) - f.g;                       // overstress; -inf if g = inf
    if (o > 0.0) {
      const double sh = sinh(f.c1 * o);
      dg = f.c0 * copysign(sh, t);
      ddg = f.c0 * f.c1 * sqrt(1.0 + sh * sh);            // cosh
    } else {
      dg = 0.0;
      ddg = 0.0;
    }
  }
}

// The power law's slip_law together with the system's potential share (slip_pot), both
// from the one power |x|^(n-1).
__device__ __forceinline__ void slip_law_pot_power(const Flow& f, double t, double& dg,
                                                   double& ddg, double& pot) {
  const double x = t * f.ig;
  const double ax = fabs(x);
  const double pw = pow_e(ax, f.c1 - 1.0, f.nm1);
  dg = f.c0 * copysign(ax * pw, x);
  ddg = f.c0 * f.c1 * f.ig * pw;
  pot = fabs(t) * ax * pw;
}

// One system's share of the dissipation potential, without the factor pot_scale:
// |t| |t/g|^n (power law), sinh(beta <|t| - g> / 2)^2 = (cosh(beta <|t| - g>) - 1) / 2
// (thermally activated; no cancellation near the threshold).
template <int F>
__device__ __forceinline__ double slip_pot(const Flow& f, double t) {
  if constexpr (F == FLOW_POWER) {
    const double ax = fabs(t * f.ig);
    return fabs(t) * ax * pow_e(ax, f.c1 - 1.0, f.nm1);
  } else {
    const double o = fabs(t) - f.g;
    if (!(o > 0.0)) return 0.0;
    const double sh = sinh(0.5 * f.c1 * o);
    return sh * sh;
  }
}
template <int F>
__device__ __forceinline__ double pot_scale(const Flow& f) {
  return F == FLOW_POWER ? f.c0 / (f.c1 + 1.0) : 2.0 * f.c0 / f.c1;
}

// Packed upper triangle of a symmetric 6x6, row-major: (0,0),(0,1)..(0,5),(1,1)..(5,5).
__device__ __forceinline__ constexpr int pk(int i, int j) {
  return (i <= j) ? i * 6 - i * (i - 1) / 2 + (j - i) : j * 6 - j * (j - 1) / 2 + (i - j);
}

// y = S x for the cubic Mandel matrix with normal block (a on, b off the diagonal) and
// shear diagonal c.
__device__ __forceinline__ void cubic_mul(double a, double b, double c, const double x[6],
                                          double y[6]) {
  y[0] = a * x[0] + b * (x[1] + x[2]);
  y[1] = a * x[1] + b * (x[0] + x[2]);
  y[2] = a * x[2] + b * (x[0] + x[1]);
  y[3] = c * x[3];
  y[4] = c * x[4];
  y[5] = c * x[5];
}

// In-place upper Cholesky J = U^T U on the packed triangle; false if not SPD.  The
// diagonal is stored inverted (1 / U_ii): the solves and the inverse then multiply where
// they would divide, and the serial chains of the triangular solves carry no divisions.
__device__ __forceinline__ bool chol6p(double J[21]) {
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = J[pk(i, i)];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= J[pk(k, i)] * J[pk(k, i)];
    if (!(s > 0.0)) return false;
    const double id = rsqrt(s);
    J[pk(i, i)] = id;
#pragma unroll
    for (int j = i + 1; j < 6; ++j) {
      double t = J[pk(i, j)];
#pragma unroll
      for (int k = 0; k < i; ++k) t -= J[pk(k, i)] * J[pk(k, j)];
      J[pk(i, j)] = t * id;
    }
  }
  return true;
}

// Solve U^T U x = b with the packed upper factor U of chol6p (inverted diagonal).
__device__ __forceinline__ void chol6p_solve(const double U[21], const double b[6], double x[6]) {
  double y[6];
#pragma unroll
  for (int i = 0; i < 6; ++i) {
    double s = b[i];
#pragma unroll
    for (int k = 0; k < i; ++k) s -= U[pk(k, i)] * y[k];
    y[i] = s * U[pk(i, i)];
  }
#pragma unroll
  for (int i = 5; i >= 0; --i) {
    double s = y[i];
#pragma unroll
    for (int k = i + 1; k < 6; ++k) s -= U[pk(i, k)] * x[k];
    x[i] = s * U[pk(i, i)];
  }
}

// K = J^-1 = U^-1 U^-T (packed 21) from the packed upper factor U of chol6p.
__device__ __forceinline__ void chol6p_inverse(const double U[21], double K[21]) {
  double W[21];            // W = U^-1, upper triangular, packed
#pragma unroll
  for (int j = 5; j >= 0; --j) {
    W[pk(j, j)] = U[pk(j, j)];
#pragma unroll
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
#pragma unroll
      for (int k = i + 1; k <= j; ++k) s += U[pk(i, k)] * W[pk(k, j)];
      W[pk(i, j)] = -s * U[pk(i, i)];
    }
  }
#pragma unroll
  for (int i = 0; i < 6; ++i)
#pragma unroll
    for (int j = i; j < 6; ++j) {
      double s = 0.0;
#pragma unroll
      for (int k = j; k < 6; ++k) s += W[pk(i, k)] * W[pk(j, k)];
      K[pk(i, j)] = s;
    }
}

__device__ __forceinline__ void sym33(const double t[6], double T[3][3]) {
  T[0][0] = t[0]; T[1][1] = t[1]; T[2][2] = t[2];
  T[1][2] = T[2][1] = t[3];
  T[0][2] = T[2][0] = t[4];
  T[0][1] = T[1][0] = t[5];
}

// Cyclic Jacobi eigen-decomposition of a symmetric 3x3 (columns of V = vectors).
__device__ inline void jacobi3(double a[3][3], double d[3], double V[3][3]) {
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) V[i][j] = (i == j) ? 1.0 : 0.0;
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = a[0][1] * a[0][1] + a[0][2] * a[0][2] + a[1][2] * a[1][2];
    const double dia = a[0][0] * a[0][0] + a[1][1] * a[1][1] + a[2][2] * a[2][2];
    if (off <= 1e-36 * dia || off == 0.0) break;
    for (int pq = 0; pq < 3; ++pq) {
      const int p = (pq == 2) ? 1 : 0;
      const int qq = (pq == 0) ? 1 : 2;
      const double apq = a[p][qq];
      if (apq == 0.0) continue;
      const double theta = (a[qq][qq] - a[p][p]) / (2.0 * apq);
      const double tt = copysign(1.0, theta) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(tt * tt + 1.0);
      const double s = tt * c;
      for (int k = 0; k < 3; ++k) {
        const double akp = a[k][p], akq = a[k][qq];
        a[k][p] = c * akp - s * akq;
        a[k][qq] = s * akp + c * akq;
      }
      for (int k = 0; k < 3; ++k) {
        const double apk = a[p][k], aqk = a[qq][k];
        a[p][k] = c * apk - s * aqk;
        a[qq][k] = s * apk + c * aqk;
      }
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][p], vkq = V[k][qq];
        V[k][p] = c * vkp - s * vkq;
        V[k][qq] = s * vkp + c * vkq;
      }
    }
  }
  d[0] = a[0][0]; d[1] = a[1][1]; d[2] = a[2][2];
}

}  // namespace rvefft
