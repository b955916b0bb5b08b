// Kernel launchers of the HIP library (host-callable, all on an explicit stream).
#pragma once
#include "common.h"

namespace rvefft {

// FFT plans of one grid: axis lengths, radix schedules and device twiddle tables.
struct Plans {
  Grid g;
  AxisPlan ax[3];
  const void* tw64[3];     // cplx<double>[n_a], exp(-2 pi i k / n_a)
  const void* tw32[3];     // cplx<float>[n_a]
  int nslot = 1;           // RVEs of a batched launch (grid z; g.sd their buffer offsets)
  const void* tw_ptr(int axis, bool f64) const { return f64 ? tw64[axis] : tw32[axis]; }
};

// Fill the constant twiddle tables of the register DFTs (current device), in every
// translation unit that holds a copy; synchronises the stream.
hipError_t upload_reg_twiddles(hipStream_t st);
hipError_t upload_reg_twiddles_zfused(hipStream_t st);

// Radix schedule of a length 2^a 3^b; returns false for other lengths.
bool make_axis_plan(int n, AxisPlan* out);

// Block-level deterministic sum: wave shuffles, then the waves in order; thread 0
// writes partial[blockIdx.x].  `red` is LDS of blockDim.x/64 doubles.
__device__ inline void block_partial_sum(double v, double* partial, double* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
    partial[blockIdx.x] = s;
  }
}

// Fixed-order sum of a[0..n) computed by every block of a kernel (so that each block
// holds the grid reduction of the previous kernel without another launch): thread t adds
// a[t], a[t + blockDim], ..., then wave shuffles and the waves in order.  Returns the same
// value to every thread of every block.  `red` is LDS of blockDim.x/64 doubles.
__device__ inline double block_sum_all(const double* __restrict__ a, int n, double* red) {
  double v = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) v += a[i];
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// Convergence test of a CG iteration, as every block of the next kernel sees it: sums
// the step's partials of <r, r> and <r, z> (2 x nb), and block 0 records <r, r> in
// sc[irr], <r, z> in sc[irz] and the flag (1 converged: <r, r> <= sc[itol2]; 2 not
// finite).  Returns true when the solve is over.  Idempotent: a second test of the same
// iteration writes the same values (the iterations are counted by the step itself).
struct CgCheck {
  const double* part;   // step partials, nullptr: no test in this kernel
  int nb, iflag, itol2, irr, irz;
};
__device__ inline bool cg_check_inline(const CgCheck& ck, double* sc, double* red, double& rz) {
  // both sums in one pass: thread-strided, wave shuffles, waves in order
  double a = 0.0, b = 0.0;
  for (int i = threadIdx.x; i < ck.nb; i += blockDim.x) {
    a += ck.part[i];
    b += ck.part[ck.nb + i];
  }
  for (int off = 32; off > 0; off >>= 1) {
    a += __shfl_down(a, off, 64);
    b += __shfl_down(b, off, 64);
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) { red[wid] = a; red[nw + wid] = b; }
  __syncthreads();
  double rr = 0.0;
  rz = 0.0;
  for (int w = 0; w < nw; ++w) { rr += red[w]; rz += red[nw + w]; }
  const bool bad = !isfinite(rr);
  const bool done = bad || rr <= sc[ck.itol2];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    sc[ck.irr] = rr;
    sc[ck.irz] = rz;
    if (bad) sc[ck.iflag] = 2.0;
    else if (done) sc[ck.iflag] = 1.0;
  }
  return done;
}

// --- spectral passes (spectral.hip) ------------------------------------------------
template <typename R>
void launch_x_r2c(const Plans& p, const void* in, bool in_f64, long long in_cs, const double* phi,
                  double kres, cplx<R>* out, long long out_cs, int ncomp, hipStream_t st,
                  const double* stop = nullptr);
template <typename R>
void launch_x_c2r(const Plans& p, const cplx<R>* in, long long in_cs, void* out, bool out_f64,
                  long long out_cs, int ncomp, double scale, int accumulate, hipStream_t st,
                  const double* stop = nullptr);
template <typename R>
void launch_x_tangent(const Plans& p, cplx<R>* data, long long cs, const R* gK, double scale,
                      hipStream_t st, const double* stop = nullptr, hipEvent_t ev0 = nullptr,
                      hipEvent_t ev1 = nullptr);
template <typename R>
void launch_fft_yz(const Plans& p, cplx<R>* data, long long cs, int ncomp, int axis, bool inv,
                   hipStream_t st, const double* stop = nullptr);
template <typename R>
void launch_sym_grad(const Plans& p, const cplx<R>* u, long long ucs, cplx<R>* e, long long ecs,
                     hipStream_t st, const double* stop = nullptr);
template <typename R>
void launch_div(const Plans& p, const cplx<R>* s, long long scs, cplx<R>* out, long long ocs,
                double sign, hipStream_t st, const double* stop = nullptr);
template <typename R>
int launch_precond(const Plans& p, const cplx<R>* r, cplx<R>* z, long long cs, const double* kbar21,
                   double* partial, hipStream_t st, const double* stop = nullptr,
                   const double* m0 = nullptr);
// Fused conjugate-gradient kernels (spectral.hip):
// p = z + (sc[ia]/sc[ib]) p, then e = sym(i xi~ (x) p)
template <typename R>
void launch_grad_cgp(const Plans& p, cplx<R>* pv, const cplx<R>* z, long long cs, const double* sc,
                     int ia, int ib, cplx<R>* e, hipStream_t st, const double* stop = nullptr);
// q = -i xi~ . s and block partials of <p, q>; returns #blocks
template <typename R>
int launch_div_dot(const Plans& p, const cplx<R>* s, cplx<R>* q, const cplx<R>* pv, long long cs,
                   double* partial, hipStream_t st, const double* stop = nullptr);
// z passes fused with the operator's end points (zfused.hip); available for even n1 and
// n3 in the register-DFT set.  zgrad_inv: p_new = z + (sc[ia]/sc[ib]) p_old (stored),
// e = F_z^-1{sym(i xi~ (x) p_new)}.  zdiv_fwd: q = -i xi~ . F_z{s} and block partials of
// <p, q>; returns #blocks.
template <typename R>
bool fused_z_available(const Plans& p);
// With ck.part set, zgrad_inv first runs the convergence test of the previous CG
// iteration (cg_check_inline) and takes beta = <r, z> / sc[ib] from it.
template <typename R>
void launch_zgrad_inv(const Plans& p, const cplx<R>* z, const cplx<R>* pold, cplx<R>* pnew,
                      long long cs, double* sc, int ia, int ib, cplx<R>* e, hipStream_t st,
                      const double* stop = nullptr, CgCheck ck = CgCheck{nullptr, 0, 0, 0, 0, 0});
template <typename R>
int launch_zdiv_fwd(const Plans& p, const cplx<R>* s, cplx<R>* q, const cplx<R>* pv, long long cs,
                    double* partial, hipStream_t st, const double* stop = nullptr);
// One CG step after the operator: alpha = sc[cur] / sc[ipq]; x += alpha p;
// z -= alpha M h(q), with h the Hermitian projection of the self-conjugate x-planes
// applied on the fly (the preconditioned residual z = M r, updated in place: M acts per
// bin, so r itself is not stored); r = M^-1 z per bin (the acoustic tensor, zero on the
// null bins where M is zero); block partials of <r, r> and <r, z> at partial[0][blk],
// partial[1][blk].  Returns #blocks.
// With pq_part set, every block first sums the nb_pq partials of <p, q> itself (and
// block 0 stores the sum in sc[ipq], the breakdown flag in sc[iflag] and counts the
// iteration in sc[iiter]); otherwise <p, q> is read from sc[ipq].  max_blocks bounds the
// grid (and so the partials).
// With m0 set (mixed macroscopic control) the zero bin holds the macro unknowns: it is
// not projected, z(0) -= alpha m0 q(0) and r(0) = m0[36..] z(0) (6 x 6 on the bin's six
// reals: m0 and its inverse on the stress-controlled block).
template <typename R>
int launch_cg_step(const Plans& p, cplx<R>* x, const cplx<R>* pv, const cplx<R>* q,
                   cplx<R>* z, long long cs, const double* kbar21, double* sc, int cur, int ipq,
                   double* partial, hipStream_t st, const double* stop,
                   const double* pq_part = nullptr, int nb_pq = 0, int iflag = 0, int iiter = 0,
                   int max_blocks = 1 << 30, const double* m0 = nullptr);
// Hermitian projection of the self-conjugate x-planes (spectra of real fields)
template <typename R>
void launch_herm_proj(const Plans& p, cplx<R>* v, long long cs, int ncomp, hipStream_t st,
                      const double* stop = nullptr);
template <typename R>
void launch_pf_scale(const Plans& p, cplx<R>* d, double ell, double scale, hipStream_t st,
                     const double* stop = nullptr, int lap = 0);
template <typename R>
void launch_curl_reg(const Plans& p, cplx<R>* b9, long long cs, double ell_fp, double scale,
                     hipStream_t st);

// --- restarted GMRES(m) vector kernels (gmres.hip) -----------------------------------------
constexpr int kGmChunk = 8;     // basis vectors per block dot / update launch
// partial[i * nblk + blk]: block sums of the Parseval-weighted <V_i, w>, i < nv <= kGmChunk,
// V_i = V + i * vs; returns nblk
template <typename R>
int launch_mdot(const Plans& p, const cplx<R>* V, long long vs, int nv, const cplx<R>* w,
                long long cs, double* partial, hipStream_t st);
// w += sign * sum_i coef[i] V_i (coef: nv <= kGmChunk device doubles)
template <typename R>
void launch_maxpy(const Plans& p, const cplx<R>* V, long long vs, int nv, const double* coef,
                  double sign, cplx<R>* w, long long cs, hipStream_t st);
// out = a in + b y (y may be null when b = 0)
template <typename R>
void launch_caxpby(const Plans& p, const cplx<R>* in, double a, const cplx<R>* y, double b,
                   cplx<R>* out, long long cs, hipStream_t st);

// --- mixed strain/stress macroscopic control (macro.hip) --------------------------------
// Six doubles passed by value to a kernel.
struct Six6 {
  double v[6];
};
// e_c += s E_c on the stress-controlled components (mask bit c, order xx yy zz yz xz xy),
// E the Mandel macro unknowns in the zero bin of pv; nz = 1: at the zero bin, nz = N3: along
// the (0, 0) z column (z still spatial, zstride apart).  de_out: (s/N) E, or nullptr.
template <typename R>
void launch_macro_strain(cplx<R>* e, long long ecs, const cplx<R>* pv, long long pcs, double s,
                         double de_scale, int mask, int nz, long long zstride, double* de_out,
                         hipStream_t st, const double* stop = nullptr);
// q(0) = s sigma^_M(0) on the stress-controlled components, and the zero-bin term of
// <p, q> at pq_out (sigma^(0): sum of the (0, 0) z column for nz = N3, the zero bin for 1).
template <typename R>
void launch_macro_stress(const cplx<R>* sg, long long scs, cplx<R>* q, const cplx<R>* pv,
                         long long cs, double s, int mask, int nz, long long zstride,
                         double* pq_out, hipStream_t st, const double* stop = nullptr);
// b(0) = -s (sigma^_M(0) - n sigma*_M) from the full spectrum of g sigma.
template <typename R>
void launch_macro_rhs(const cplx<R>* sg, long long scs, cplx<R>* b, long long cs, double s,
                      double n, const double tgt[6], int mask, hipStream_t st);
// m0[0..36) = (s2 Kbar_FF)^-1 and m0[36..72) = s2 Kbar_FF (6 x 6 each, zero outside the
// stress-controlled block)
void launch_macro_prec(const double* kbar21, double s2, int mask, double* m0, hipStream_t st);

// --- voxel kernels (voxel.hip) -------------------------------------------------------
// Per-grain table: GT_STRIDE doubles per grain.
enum {
  GT_C = 0,        // Mandel stiffness, 36 (sample frame)
  GT_S = 36,       // Mandel compliance, 36
  GT_P = 72,       // Mandel Schmid tensors sym(s (x) n), 12 x 6
  GT_SN = 144,     // s (x) n, 12 x 9 row-major
  GT_R = 252,      // rotation crystal -> sample, 9 row-major
  GT_TAU0 = 261,   // initial critical resolved shear stress
  GT_STRIDE = 262
};

// Grain-independent crystal-frame constants (Mandel): Schmid tensors of the 12 slip
// systems, cubic stiffness (c11, c12 normal block, c66 = 2 C44 shear) and its inverse.
struct CrystalFrame {
  double P[72];
  double c11, c12, c66, s11, s12, s66;
};

// Flow rules: power law dgamma = dt gdot0 sign(tau) |tau/g|^n (linear hardening), or
// thermally activated glide dgamma = dt A sign(tau) sinh(beta <|tau| - g>) with
// A = rho_m b^2 v_D exp(-dF/kT), beta = dV/kT (eq. flowrule; Taylor hardening).
enum { FLOW_POWER = 0, FLOW_DUNNE = 1 };

struct Material {
  double dt, gdot0, nexp, kres, h_lin, lambda_ssd, xi_store, G_crit, ell, Gc, burgers;
  int nexp_int;   // nexp when it is an integer in [1, 64], else 0 (then pow is used)
  int flow;       // FLOW_POWER or FLOW_DUNNE
  double A, beta; // thermally activated rule: rate prefactor [1/s], dV/kT [1/Pa]
  double mu_b;    // Taylor hardening: shear modulus times Burgers vector [Pa m]
};

// number of reduction values written by each voxel kernel per block
enum { RED_CONST = 28,  // 21 sum gK, 1 sum g*w, 6 sum g*sigma
       RED_SOURCE = 2,  // sum S, sum S^2
       RED_COMMIT = 15, // 6 sum g*sigma, 6 sum eps, max phi, n_trig, max phi outside pre-set
       RED_MAX4 = 4 };

int voxel_grid(long long n);

// Returns the number of block partials written (RED_CONST components, component-major) for
// launch_reduce: one per 256-voxel block of the return map, whose kernel forms them, or, with
// plane stress (the sums follow the condensation), those of a separate pass.
template <typename R>
int launch_constitutive(long long N, const double* eps, const double* deps, double t,
                        const double* epsp, const double* gslip, const int* grain,
                        const double* gtab, double* sig, const double* phi, R* gK, double* gw,
                        const CrystalFrame& cf, const Material& m, double* partial, int* fail,
                        hipStream_t st, double* ps_sig = nullptr, double* ps_rec = nullptr);
// plane stress: d e_O = -B d e_P - r on the Newton correction, from the per-voxel B and r
// that the constitutive launch's condensation left in rec (12 N)
void launch_plane_recover(long long N, double* deps, const double* rec, hipStream_t st);
void launch_source(long long N, const double* eps, const double* sig, const double* epsp,
                   const double* gslip, const int* grain, const double* gtab, const double* wp,
                   const double* trig, const double* wcrit, double* S, double* wep,
                   const Material& m, double* partial, hipStream_t st);
// GND-coupled hardening (option): end-of-increment plastic distortion (9) and SSD density
// of the slip at the converged stress and the current strength
void launch_trial_hardening(long long N, const double* sig, const double* gslip,
                            const double* beta, const double* rho_ssd, const int* grain,
                            const double* gtab, const Material& m, double* beta_tr,
                            double* rho_ssd_tr, hipStream_t st);
// g_next = tau_c0 + mu b sqrt(rho_SSD + rho_GND) of those densities; partial maxima of
// |g_next - g| and |g_next - g_n| (2 values) over the voxels that can slip
void launch_taylor_next(long long N, const double* gslip, const double* g_n,
                        const double* rho_ssd_tr, const double* rho_gnd_tr, const int* grain,
                        const double* gtab, double mu_b, double* g_next, double* partial,
                        hipStream_t st);
// Aitken's delta-squared relaxation of the coupled strength's fixed point g = T(g) (Irons
// and Tuck), over the voxels that can slip, with r = g_next - g the pass's residual:
// partial sums of r_prev . (r - r_prev) and |r - r_prev|^2 (2 values; r_prev read as 0 on
// the first pass), then g <- g + omega r and r_prev <- r
void launch_aitken_dots(long long N, const double* gslip, const double* g_next,
                        const double* r_prev, int first, double* partial, hipStream_t st);
void launch_aitken_relax(long long N, double* gslip, const double* g_next, double* r_prev,
                         double omega, hipStream_t st);
// Taylor hardening g = tau_c0 + mu b sqrt(rho_SSD + rho_GND) of the voxels that can slip
void launch_taylor(long long N, double* gslip, const double* rho_ssd, const double* rho_gnd,
                   const int* grain, const double* gtab, double mu_b, hipStream_t st);
void launch_commit(long long N, const double* sig, double* gslip, double* epsp, double* beta,
                   double* rho_ssd, const double* rho_gnd, double* wp, double* gs, double* H,
                   double* wcrit, double* trig, const double* wep, const double* phi,
                   const double* eps, const int* grain, const double* gtab, const Material& m,
                   double* partial, hipStream_t st);
void launch_gnd(long long N, const double* lam9, const int* grain, const double* gtab,
                const double* Q81, double burgers, double* rho_gnd, hipStream_t st);
// eps += t * deps; partial maxima of |t deps| and |eps - eps_t| (2 values)
void launch_eps_update(long long N, double* eps, const double* deps, double t, const double* eps_t,
                       double* partial, hipStream_t st);
// partial sum of g(phi) sigma : deps (tensor double contraction)
void launch_slope(long long N, const double* sig, const double* deps, const double* phi,
                  double kres, double* partial, hipStream_t st);
// staggered-loop maxima: |eps-eps_prev|, |eps-eps_t|, |phi-phi_prev|, |phi-phi_t|
void launch_stag_norms(long long N, const double* eps, const double* eps_prev, const double* eps_t,
                       const double* phi, const double* phi_prev, const double* phi_t,
                       double* partial, hipStream_t st);
// eps[c] += de[c] for the 6 components (uniform macroscopic increment)
void launch_add_uniform(long long N, double* eps, const double de[6], hipStream_t st);
// phi = min(1, max(phi_t, x))
void launch_clamp(long long N, const double* x, const double* phi_t, double* phi, hipStream_t st);
// out = g(phi) sig on 6 components (the degraded stress), g(phi) = (1 - phi)^2 + kres
void launch_degrade(long long N, const double* sig, const double* phi, double kres, double* out,
                    hipStream_t st);
// Phase field with the pre-set crack (voxels with an infinite slip resistance) held at 1
// (pfdir.hip).  mode 0: y = P x;  1: y = 1 - P 1 (the indicator of the crack);
// 2: y = P ((1 + 2S) x + w);  3: y = P (2S - ((1 + 2S) x + w)); P the restriction to the
// free voxels.  Each is a no-op once *stop is non-zero.
void launch_pfd(long long N, int mode, const double* x, const double* w, const double* S,
                const double* gslip, double* y, hipStream_t st, const double* stop = nullptr);
// y += a x  (a = sign * sc[ia] / sc[ib] when sc is set, else a = sign)
void launch_pfd_axpy(long long N, const double* sc, int ia, int ib, double sign, const double* x,
                     double* y, hipStream_t st, const double* stop = nullptr);
// p = z + (sc[ia] / sc[ib]) p
void launch_pfd_xpby(long long N, const double* z, const double* sc, int ia, int ib, double* p,
                     hipStream_t st, const double* stop = nullptr);

// --- finite-strain kinematics (finite.hip) --------------------------------------------------
// Crystal-frame slip directions s_a and plane normals n_a (12 x 3 each, unit) and the cubic
// Mandel stiffness / compliance constants.
struct FsFrame {
  double s[36], n[36];
  double c11, c12, c66, s11, s12, s66;
};
struct Nine9 {
  double v[9];
};
// Return map, first Piola-Kirchhoff stress, trial plastic deformation, 9 x 9 degraded
// tangent and the per-voxel increments aux = (sum tau dgamma, sum |dgamma|, dLp : dLp,
// W_e+) at F + t dF (dF may be null); Sws (crystal-frame S, 6) is the warm start, updated.
void launch_fs_constitutive(long long N, const double* F, const double* dF, double t,
                            const double* Fpn, const double* gslip, const int* grain,
                            const double* gtab, double* Sws, const double* phi, double* P,
                            double* fp_tr, double* aux, double* gK, const FsFrame& fr,
                            const Material& m, int* fail, hipStream_t st);
// e_ij = i xi~_j u_i (3 -> 9 half-spectrum components)
void launch_fs_grad(const Plans& p, const cplx<double>* u, long long ucs, cplx<double>* e,
                    long long ecs, hipStream_t st, const double* stop = nullptr);
// out_i = sign i xi~_j s_ij (9 -> 3)
void launch_fs_div(const Plans& p, const cplx<double>* s, long long scs, cplx<double>* out,
                   long long ocs, double sign, hipStream_t st, const double* stop = nullptr);
// z = [xi~ . Kbar . xi~]^-1 P r, Kbar the 81-entry mean tangent (device), P the Hermitian
// projection of the self-conjugate x-planes
void launch_fs_precond(const Plans& p, const cplx<double>* r, cplx<double>* z, long long cs,
                       const double* kbar81, hipStream_t st, const double* stop = nullptr);
// x <- gK : x on 9 real components per voxel (in place)
void launch_fs_tangent(double* x, long long N, const double* gK, hipStream_t st,
                       const double* stop = nullptr);
// block sums of every component of an ncomp x N field: partial[c * nb + b]; returns nb
int launch_colsum(const double* x, long long N, int ncomp, double* partial, hipStream_t st);
void launch_fs_add_uniform(long long N, double* F, const double d[9], hipStream_t st);
// F += t dF; partial maxima of |t dF| and |F - F_t| (2 values)
void launch_fs_update(long long N, double* F, const double* dF, double t, const double* Ft,
                      double* partial, hipStream_t st);
// maxima |F - F_prev|, |F - F_t|, |phi - phi_prev|, |phi - phi_t|
void launch_fs_stag_norms(long long N, const double* F, const double* Fprev, const double* Ft,
                          const double* phi, const double* phi_prev, const double* phi_t,
                          double* partial, hipStream_t st);
void launch_fs_source(long long N, const double* aux, const double* wp, const double* trig,
                      const double* wcrit, double* S, const Material& m, double* partial,
                      hipStream_t st);
// partials: 19 sums (9 g(phi) P, 9 F, n_trig) then 2 maxima (phi, phi where slip is possible)
void launch_fs_commit(long long N, const double* P, const double* F, double* Fp,
                      const double* fp_tr, double* gslip, double* rho_ssd, const double* rho_gnd,
                      double* wp, double* gs, double* H, double* wcrit, double* trig,
                      const double* aux, const double* phi, const Material& m, double* partial,
                      hipStream_t st);
// out = g(phi) P on 9 components
void launch_fs_degrade(long long N, const double* P, const double* phi, double kres, double* out,
                       hipStream_t st);

// --- reductions and vector kernels (vector.hip) ---------------------------------------
// out[c] = sum (or max) over b < nblk of partial[c*nblk + b], fixed order.
// CG reductions with the device-side control: reduce_pq sums the partials of <p, q>
// into sc[ipq] and sets sc[iflag] = 2 unless it is positive and finite; reduce_check
// sums <r, r> and <r, z>, counts the iteration in sc[iiter], stores <r, z> in sc[nxt] and
// <r, r> in sc[irr], and sets sc[iflag] to 1 when <r, r> <= sc[itol2] or 2 when it is not
// finite.  Both are no-ops once sc[iflag] is non-zero.
void launch_reduce_pq(const double* partial, int nblk, double* sc, int ipq, int iflag,
                      hipStream_t st);
// cg_check_inline in one block (the test of a batch's last iteration); no-op once
// sc[ck.iflag] is non-zero
void launch_cg_check_tail(double* sc, const CgCheck& ck, hipStream_t st,
                          const long long* sd = nullptr, int nslot = 1);
void launch_reduce_check(const double* partial, int nblk, double* sc, int iiter, int nxt, int irr,
                         int iflag, int itol2, hipStream_t st);
void launch_reduce(const double* partial, int nblk, int ncomp, int op_max, double* out,
                   hipStream_t st, const double* stop = nullptr);
// Parseval-weighted <a,b> over ncomp half-spectrum components; returns #blocks.
template <typename R>
int launch_sdot(const Plans& p, const cplx<R>* a, const cplx<R>* b, long long cs, int ncomp,
                double* partial, hipStream_t st, const double* stop = nullptr);
// real-vector kernels (phase field); every one is a no-op once *stop is non-zero
int launch_rdot(long long n, const double* a, const double* b, double* partial, hipStream_t st,
                const double* stop = nullptr);
// pq = <p, w + 2 S p>
int launch_pf_pq(long long n, const double* p, const double* w, const double* S, double* partial,
                 hipStream_t st, const double* stop = nullptr);
// x += a p ; r -= a (w + 2 S p) ; partial <r,r>
int launch_pf_xr(long long n, double* x, double* r, const double* p, const double* w,
                 const double* S, const double* sc, int ia, int ib, double* partial, hipStream_t st,
                 const double* stop = nullptr);
// p = z + b p ; w = r + b w
void launch_pf_pw(long long n, double* p, double* w, const double* z, const double* r,
                  const double* sc, int ia, int ib, hipStream_t st, const double* stop = nullptr);
// convergence test of a phase-field CG iteration (flag as launch_reduce_check): counts the
// iteration in sc[iiter], sets sc[iflag] to 2 unless sc[ipq] > 0 and sc[irr] is finite, else
// to 1 when sc[irr] <= sc[itol2]
void launch_pf_check(double* sc, int iflag, int iiter, int ipq, int irr, int itol2,
                     hipStream_t st);
// y = a * x (real)
void launch_rscale(long long n, const double* x, double a, double* y, hipStream_t st);
// zero a complex/real buffer of `bytes` bytes with a fill kernel
void launch_zero(void* ptr, size_t bytes, hipStream_t st);

}  // namespace rvefft
