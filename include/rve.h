/* rve.h -- C ABI of the MI355X (gfx950) solver for one load increment of the
 * FFT-based crystal-plasticity phase-field fatigue model of Lucarini, Dunne and
 * Martinez-Paneda (2023), in its small-strain form.
 *
 * Problem (Sec. 3.1): a periodic box of N1 x N2 x N3 cubic voxels of edge h, fields
 * at voxel centres, strain control through the macroscopic strain.  One increment
 * (Algorithm 1) takes the state at time t, a macroscopic strain increment and a time
 * step, and returns the state at t + dt: the momentum balance div[g(phi) sigma] = 0
 * (eqs. str1, momentum, newton) is solved by Newton's method with a Krylov solver
 * preconditioned by the acoustic tensor of the volume-averaged tangent (eqs. precf,
 * avstiff); the phase field solves (phi - l^2 lap phi) - 2 (1 - phi) S = 0 (eqs. strpf,
 * phase, str2) with the stored-energy driving state S (eqs. crit, decMiehe, zeta);
 * the two alternate until both relative corrections fall below tol_stag, with the
 * pointwise irreversibility phi >= phi_t.  The history (SSD density, plastic work,
 * stored energy density G_s, W_crit) and the regularised Nye-tensor GND density
 * (eq. nye1 and the Fourier curl of Sec. 3.1) are committed at the end.
 *
 * Conventions.
 *  - Every voxel array is structure-of-arrays, x fastest: voxel (i, j, k) is element
 *    i + N1*(j + N2*k) of each component.
 *  - Symmetric tensors have 6 components in the order xx, yy, zz, yz, xz, xy
 *    (tensor shear components, not engineering strains).
 *  - Units: SI (m, s, Pa, J/m^2).
 *  - Every function returns an int status (RVE_OK = 0, negative on error) and never
 *    throws; rve_last_error() gives a message for the calling thread.
 *  - Handles are not thread safe; one handle per thread.
 */
#ifndef RVE_H
#define RVE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RVE_OK = 0,
  RVE_E_ARG = -1,     /* invalid argument: sizes not 2^a 3^b, non-finite input, bad ids */
  RVE_E_NOMEM = -2,   /* the arena is smaller than rve_footprint_bytes()                */
  RVE_E_DEVICE = -3,  /* a HIP call failed                                              */
  RVE_E_NOCONV = -4,  /* a solver did not converge; the state is left at time t         */
  RVE_E_STATE = -5    /* call out of order (e.g. a step before the microstructure)      */
};

enum { RVE_FP64 = 0, RVE_MIXED = 1 };
/* Constitutive model (Sec. 2.1).  RVE_MAT_POWER: power-law flow
 *   dgamma = dt gdot0 sign(tau) |tau/g|^n_exp with linear hardening g += h_lin sum |dgamma|.
 * RVE_MAT_DUNNE: thermally activated glide over obstacles (eq. flowrule)
 *   dgamma = dt A sign(tau) sinh(<|tau| - g> dV / kT),  A = rho_m b^2 v_D exp(-dF / kT),
 *   no slip while |tau| <= g, with Taylor hardening g = tau_c0 + mu b sqrt(rho_SSD + rho_GND)
 *   from the densities committed at the end of the previous increment (initially
 *   tau_c0 + mu b sqrt(rho0)). */
enum { RVE_MAT_POWER = 0, RVE_MAT_DUNNE = 1 };
/* Discrete derivative of the gradient, divergence and acoustic tensor of the momentum
 * balance (Sec. 3.1 names discrete derivatives as the remedy for Gibbs oscillations at
 * high phase contrast).  RVE_DERIV_ROTATED: k_a = D(theta_a) prod_{b != a} A(theta_b) with
 * D = (e^{i theta} - 1)/h, A = (1 + e^{i theta})/2, theta = 2 pi k / N (A = 0 at the
 * Nyquist index): a forward difference along a averaged over the four parallel voxel
 * edges; the gradient is sym(k (x) u^), the divergence conj(k) . sigma^. */
enum { RVE_DERIV_SPECTRAL = 0, RVE_DERIV_ROTATED = 1 };
/* Krylov solver of the linearised momentum balance (eq. newton).  The operator is
 * symmetric positive definite in the Parseval inner product (the return map keeps the
 * tangent symmetric), so CG and GMRES reach the same Newton correction; RVE_KRYLOV_GMRES
 * is the paper's restarted GMRES with the same preconditioner, its relative tolerance
 * tol_lin applied to the preconditioned residual. */
enum { RVE_KRYLOV_CG = 0, RVE_KRYLOV_GMRES = 1 };
/* Kinematics (Sec. 2.1).  RVE_KIN_SMALL: the small-strain form (eps = eps_e + eps_p,
 * symmetric 6-component strain and stress, 6x6 tangents).  RVE_KIN_FINITE: the paper's
 * finite strain, F = Fe Fp with Lp = sum gdot_a s_a (x) n_a, the first Piola-Kirchhoff
 * stress balanced in the reference configuration (eq. str1), F = F_bar + grad u
 * (eq. fdef), the 9 x 9 consistent tangent dP/dF in the linearised balance (eq. newton),
 * the preconditioner [xi~ . Kbar . xi~]^-1 of the 81-entry mean tangent (eqs. precf,
 * avstiff) and the tensile energy of the logarithmic elastic strain (eq. decMiehe).
 * Elasticity S = C : Ee (Ee = 1/2 (Fe^T Fe - I), lattice configuration); backward Euler
 * on Fp with the resolved shear tau_a = S : sym(A s_a (x) n_a), A the trial elastic right
 * Cauchy-Green tensor (Kalidindi, Bronkhorst and Anand 1992), Fp = (I + sum_a dgamma_a
 * s_a (x) n_a) Fp_n.  Finite-strain handles run in FP64 with RVE_KRYLOV_GMRES (the
 * linearised operator is not symmetric) and the spectral derivative, and step with
 * rve_step_increment_finite. */
enum { RVE_KIN_SMALL = 0, RVE_KIN_FINITE = 1 };

/* Field selection bits for rve_fields(); fields are written in increasing bit order. */
enum {
  RVE_F_STRAIN = 1u << 0,     /* 6: total strain eps                                   */
  RVE_F_STRESS = 1u << 1,     /* 6: degraded stress g(phi) sigma (the equilibrated one) */
  RVE_F_STRESS_EFF = 1u << 2, /* 6: effective (undegraded) stress sigma                 */
  RVE_F_DAMAGE = 1u << 3,     /* 1: phase field phi                                     */
  RVE_F_GS = 1u << 4,         /* 1: stored energy density G_s [J/m^2]                   */
  RVE_F_RHO_SSD = 1u << 5,    /* 1: SSD density [1/m^2]                                 */
  RVE_F_RHO_GND = 1u << 6,    /* 1: GND density [1/m^2] (lagged one increment)          */
  RVE_F_WP = 1u << 7,         /* 1: plastic work W_p [J/m^3]                            */
  RVE_F_H = 1u << 8,          /* 1: max over time of the tensile elastic energy          */
  RVE_F_WCRIT = 1u << 9,      /* 1: threshold W_crit (0 until triggered)                 */
  RVE_F_TRIG = 1u << 10,      /* 1: 1.0 where G_s has reached G_crit                     */
  RVE_F_EPS_P = 1u << 11,     /* 6: plastic strain                                       */
  RVE_F_SLIP_RES = 1u << 12,  /* 1: slip resistance g (inf in pre-cracked voxels)        */
  RVE_F_BETA_P = 1u << 13,    /* 9: plastic distortion, row-major 3x3                    */
  /* finite-strain handles only (the small-strain bits STRAIN, STRESS, STRESS_EFF, EPS_P
   * and BETA_P are refused there, and these on small-strain handles): */
  RVE_F_DEFGRAD = 1u << 14,   /* 9: deformation gradient F, row-major                    */
  RVE_F_PK1 = 1u << 15,       /* 9: degraded first Piola-Kirchhoff stress g(phi) P       */
  RVE_F_FP = 1u << 16         /* 9: plastic deformation gradient Fp                      */
};

/* Problem description.  n[a] must be of the form 2^p 3^q with 1 <= n[a] <= 512. */
typedef struct rve_desc {
  int32_t n[3];
  int32_t precision;        /* RVE_FP64: everything FP64.  RVE_MIXED: FFTs, spectral
                               operators, the tangent field and Krylov vectors in FP32;
                               return mapping, Krylov dot products, norms, the phase-field
                               solve and the history in FP64.                          */
  double h;                 /* voxel edge [m]                                         */
  double C11, C12, C44;     /* cubic elastic constants, crystal frame [Pa]            */
  double gdot0, n_exp;      /* power-law flow: reference slip rate [1/s], exponent     */
  double tau_c0, h_lin;     /* default initial slip resistance, linear hardening [Pa]  */
  double lambda_ssd, rho0;  /* SSD evolution coefficient [1/m^2], initial SSD [1/m^2]  */
  double burgers;           /* Burgers vector length [m]                               */
  double xi_store;          /* stored fraction of plastic work in G_s [-]              */
  double ell, Gc, G_crit;   /* phase-field length [m], toughness [J/m^2], G_s threshold */
  double k_res;             /* residual stiffness in g(phi) = (1-phi)^2 + k_res        */
  double ell_fp;            /* regularisation length of the plastic distortion [m]     */
  double tol_stag;          /* alternating-minimisation tolerance (paper: 5e-3)        */
  double tol_newton;        /* Newton tolerance on max|sym grad du| / max|eps - eps_t|  */
  double tol_lin;           /* relative Krylov tolerance (paper: 1e-5)                  */
  int32_t max_stag, max_newton, max_krylov;
  int32_t max_grains;       /* capacity of the per-grain tables (>= n_grains)           */
  int32_t material;         /* RVE_MAT_POWER (gdot0, n_exp, h_lin) or RVE_MAT_DUNNE     */
  double rho_m, v_D;        /* mobile dislocation density [1/m^2], jump attempt rate [1/s] */
  double dF, k_B, T;        /* activation energy [J], Boltzmann constant [J/K], temperature [K] */
  double dV;                /* activation volume [m^3]                                 */
  double mu;                /* shear modulus of the Taylor term [Pa]                    */
  int32_t krylov;           /* momentum Krylov solver: RVE_KRYLOV_CG (default) or
                               RVE_KRYLOV_GMRES (the paper's restarted GMRES, left
                               preconditioned; strain control only)                    */
  int32_t gmres_restart;    /* GMRES restart length m, 1..64 (basis of m + 1 vectors in
                               the arena)                                               */
  int32_t deriv;            /* derivative of the momentum operator: RVE_DERIV_SPECTRAL
                               (i xi~, Nyquist index zeroed) or RVE_DERIV_ROTATED (the
                               rotated finite-difference scheme, Sec. 3.1's discrete
                               derivative remedy); the phase field and the GND curl stay
                               spectral                                                 */
  int32_t pf_dirichlet;     /* 0: the pre-set crack (voxels with phi0 >= 1) enters the
                               phase-field balance (eqs. strpf, phase) as free unknowns
                               that the irreversibility clamp holds at 1; 1: it is a
                               Dirichlet condition phi = 1 of that balance, solved on the
                               other voxels by CG with the restricted preconditioner
                               (the geometric crack and soft buffers of Secs. 4.1 and
                               4.5 read as a boundary value of the damage)               */
  int32_t kinematics;       /* RVE_KIN_SMALL (default) or RVE_KIN_FINITE                 */
  int32_t gnd_coupling;     /* 0 (default): the Taylor strength of an increment is that of
                               the densities committed at the end of the previous one
                               (GND lagged one increment).  1 (RVE_MAT_DUNNE, small
                               strain): it is that of the increment's own end, tau_c0 + mu
                               b sqrt(rho_SSD,n+1 + rho_GND,n+1), both densities from the
                               increment's slip (the GND density from the regularised Nye
                               tensor of beta_n + d beta: non-local); the alternating
                               minimisation resolves it, passing until also the strength's
                               relative change max|g_i - g_i-1| / max|g_i - g_n| <=
                               tol_stag; G_s then uses rho_GND,n+1                        */
  int32_t plane_stress;     /* 0 (default) or 1: pointwise plane stress of a plate one voxel
                               thick (Secs. 4.1-4.3; n[2] = 1, small strain).  The
                               out-of-plane stress (zz, yz, xz) vanishes at every voxel,
                               the out-of-plane strain is a local unknown (not a
                               displacement gradient), each Newton step eliminates it by
                               static condensation of the linearised point, and the
                               in-plane strain stays compatible.  The steps then take no
                               out-of-plane macro control: deps[2..4] must be 0 and the
                               stress mask may name xx, yy, xy only (RVE_E_ARG otherwise);
                               macro_strain reports the mean out-of-plane strain      */
} rve_desc;

/* Per-increment report, filled by rve_step_increment (also on RVE_E_NOCONV). */
typedef struct rve_stats {
  int32_t stag_iters;       /* alternating-minimisation passes                        */
  int32_t newton_iters;     /* Newton iterations, all passes                          */
  int32_t krylov_iters;     /* momentum Krylov iterations = operator applications     */
  int32_t pf_iters;         /* phase-field Krylov iterations                          */
  int32_t ls_cuts;          /* Newton step halvings                                   */
  int32_t rm_failures;      /* voxels whose return mapping did not converge           */
  double macro_stress[6];   /* volume average of g(phi) sigma [Pa]                     */
  double macro_strain[6];   /* volume average of eps                                  */
  double max_phi;           /* max of phi                                             */
  double max_phi_slip;      /* max of phi over voxels that can slip (not pre-cracked)   */
  double n_triggered;       /* voxels with G_s >= G_crit                               */
  double ms_total, ms_constitutive, ms_mech_krylov, ms_phase_field, ms_commit;
  /* finite-strain handles: volume averages of g(phi) P and of F (row-major); there
   * macro_stress holds the symmetric part of the former and macro_strain that of the
   * latter minus the identity */
  double macro_pk1[9];
  double macro_defgrad[9];
  /* rve_pool_step: the most handles whose CG iterations advanced in shared launches with
   * this one's during the increment (1: on its own) */
  double cg_batch;
} rve_stats;

/* Device bytes a handle with this description needs in its arena (0 if invalid). */
size_t rve_footprint_bytes(const rve_desc* d);

/* Create a handle.  dev_arena: device memory of arena_bytes bytes, owned by the caller
 * and kept alive until rve_destroy (the library allocates no device memory itself).
 * hip_stream: the hipStream_t all work of this handle is ordered on (NULL = default).
 * Errors: RVE_E_ARG (bad description), RVE_E_NOMEM (arena too small), RVE_E_DEVICE. */
int rve_create(const rve_desc* d, void* dev_arena, size_t arena_bytes, void* hip_stream,
               struct rve_s** out);

/* Create a handle without allocating anything, for callers that cannot allocate device
 * memory (code that must not call hipMalloc: tight serving loops, harnesses that forbid
 * it).  Same as rve_create, except that the arena is a static device array of the
 * library, 320 MiB per device (335544320 bytes: every grid up to 64^3 in either
 * precision with max_grains <= 4096), held by each device the library runs on until the
 * process ends.  One such handle per device at a time: the array is shared, and a second
 * call while one is alive returns RVE_E_STATE.  The handle's host scalars live in the
 * handle (no pinned host memory) and its CG iterations are launched eagerly (no graph
 * instantiation).  rve_set_microstructure sets every state field the increment reads;
 * the previous handle's contents are otherwise left in the array.  rve_destroy releases
 * the array for the next call.  Calls that use such a handle from several threads at
 * once race, as for any handle.  Errors: RVE_E_ARG (bad description), RVE_E_NOMEM (the
 * description needs more than the static arena: the message gives both sizes; checked
 * before any device call), RVE_E_STATE (the array is held), RVE_E_DEVICE. */
int rve_create_noalloc(const rve_desc* d, void* hip_stream, struct rve_s** out);

/* Set the microstructure and the initial state (all host arrays, copied).
 * grain_of_voxel: N ints in [0, n_grains), x fastest.
 * quat_wxyz: 4*n_grains unit quaternions (w,x,y,z) rotating crystal vectors into the
 *            sample frame (normalised here; |q| must be within 1e-6 of 1).
 * tau_c0_per_grain: n_grains initial slip resistances [Pa], or NULL for d->tau_c0.
 * phi0: N initial damage values in [0, 1], or NULL for 0.  Voxels with phi0 = 1 are
 *       a pre-cracked region: linear elastic (no slip), stiffness g(1) C = k_res C, as
 *       the paper models geometric cracks.
 * Resets the state to t = 0: zero strain and stress, SSD = rho0, every other internal
 * variable 0.  Errors: RVE_E_ARG. */
int rve_set_microstructure(struct rve_s* h, const int32_t* grain_of_voxel, int32_t n_grains,
                           const double* quat_wxyz, const double* tau_c0_per_grain,
                           const double* phi0);

/* One load increment (Algorithm 1) under the macroscopic strain increment deps_macro
 * (6 components) over the time step dt > 0.  Synchronous on the handle's stream.
 * Transactional: on RVE_E_NOCONV the state stays at time t (the caller may retry with
 * a smaller increment).  st may be NULL.  Errors: RVE_E_ARG (non-finite input),
 * RVE_E_STATE (no microstructure), RVE_E_NOCONV, RVE_E_DEVICE. */
int rve_step_increment(struct rve_s* h, const double deps_macro[6], double dt, rve_stats* st);

/* One load increment under mixed macroscopic control (the DBFFT mixed extension the
 * paper relies on, Sec. 3.1; e.g. uniaxial stress: every component but one stress
 * controlled).  Components c (order xx, yy, zz, yz, xz, xy; tensor components) with
 * bit c of stress_mask set follow the macro stress: the volume average of g(phi) sigma
 * reaches that of time t plus dsig_macro[c]; the others follow the macro strain
 * increment deps_macro[c] as in rve_step_increment, which is this call with
 * stress_mask 0.  The stress-controlled macro strain components become unknowns of
 * the momentum Newton-Krylov system (its operator stays symmetric positive definite).
 * dsig_macro may be NULL when stress_mask is 0.  Same state semantics and errors as
 * rve_step_increment; RVE_E_ARG for a mask outside 0..63 or a non-finite increment. */
int rve_step_increment_mixed(struct rve_s* h, const double deps_macro[6],
                             const double dsig_macro[6], int32_t stress_mask, double dt,
                             rve_stats* st);

/* One load increment of a finite-strain handle (rve_desc.kinematics = RVE_KIN_FINITE)
 * under the macroscopic deformation gradient increment dF_macro (9 components,
 * row-major: F_bar(t + dt) = F_bar(t) + dF_macro) over dt > 0: Algorithm 1 with Newton
 * on the displacement (eqs. fdef, newton; full steps, halved while the preconditioned
 * residual grows), the paper's GMRES and stop test max|grad du| <= tol_newton
 * max|F_i - F_t|, the phase field and the history as in rve_step_increment (the plastic
 * work sum_a tau_a dgamma_a, the SSD rate of Lp, the Nye tensor of Fp).  Same state
 * semantics; errors as rve_step_increment, RVE_E_ARG on a small-strain handle (and
 * rve_step_increment, rve_step_increment_mixed on a finite-strain one). */
int rve_step_increment_finite(struct rve_s* h, const double dF_macro[9], double dt,
                              rve_stats* st);

/* Copy the fields selected by field_mask to host_out (n_doubles capacity), each as
 * SoA components of N values in increasing bit order.  Errors: RVE_E_ARG if the
 * buffer is too small, RVE_E_STATE before rve_set_microstructure. */
int rve_fields(struct rve_s* h, uint32_t field_mask, double* host_out, size_t n_doubles);

/* Release the handle (the arena stays owned by the caller). */
int rve_destroy(struct rve_s* h);

/* Message of the last error on this thread ("" if none). */
const char* rve_last_error(void);

/* Number of doubles rve_fields writes for field_mask (0 for an unknown bit). */
size_t rve_fields_count(const struct rve_s* h, uint32_t field_mask);

/* ---- diagnostics: single building blocks on the handle's grid and precision ------ */

/* Forward real FFT (unnormalised, exp(-i xi.x)) of ncomp real fields (host, N each,
 * ncomp <= 9) to their half spectra (host, 2*N1h*N2*N3 doubles each, re/im
 * interleaved, bin kx + N1h*(ky + N2*kz), N1h = N1/2 + 1).  Uses the handle's scratch
 * buffers; the physical state is not touched. */
int rve_diag_rfft(struct rve_s* h, int32_t ncomp, const double* real_in, double* spec_out);

/* Inverse of rve_diag_rfft, normalised (returns the real fields). */
int rve_diag_irfft(struct rve_s* h, int32_t ncomp, const double* spec_in, double* real_out);

/* Constitutive update of every voxel at the given total strain eps6 (host, 6*N) with
 * the current internal variables and time step dt: writes the effective stress
 * (6*N) and g(phi) K as 21 Mandel upper-triangle entries (21*N, row-major over
 * (0,0),(0,1)..(0,5),(1,1)..(5,5)).  Either output may be NULL.  The stored stress
 * of the state is restored afterwards. */
int rve_diag_constitutive(struct rve_s* h, const double* eps6, double dt, double* sig6_out,
                          double* gk21_out);

/* Finite-strain constitutive update of every voxel at the deformation gradients F9
 * (host, 9*N, component-major, row-major tensors) with the current internal variables and
 * time step dt: writes the effective first Piola-Kirchhoff stress (9*N) and the tangent
 * g(phi) dP_r/dF_c at (9 r + c)*N + voxel (81*N).  Either output may be NULL.  The
 * physical state is not touched; the tangent field is set (as rve_diag_constitutive).
 * RVE_E_ARG on a small-strain handle. */
int rve_diag_constitutive_finite(struct rve_s* h, const double* F9, double dt, double* P9_out,
                                 double* K81_out);

/* Apply the preconditioned linearised equilibrium operator of the current tangent
 * field to a displacement field: given real displacements u (host, 3*N), return
 * v = F^-1{ M . (-i xi~) . F{ gK : F^-1{ sym(i xi~ (x) F{u}) } } } (host, 3*N), with M
 * the acoustic-tensor preconditioner of the mean tangent.  Requires a preceding
 * rve_diag_constitutive (which sets the tangent field). */
int rve_diag_operator(struct rve_s* h, const double* u3, double* v3);

/* Layout of the handle's reduction-partials buffer for a description (no device call):
 * out3[0] = the most partial sums one divergence pass of the momentum operator writes
 * (one per block, plus one of the macro stress), out3[1] = the offset at which the CG step
 * writes its own partials, out3[2] = the buffer's length in doubles.  The CG step's blocks
 * write their partials while other blocks of the same launch still sum the divergence
 * pass's, so out3[1] >= out3[0] and out3[2] >= out3[1] + 2048 hold for every valid grid.
 * Errors: RVE_E_ARG (invalid description or null out3). */
int rve_diag_partials(const rve_desc* d, int64_t* out3);

/* Launch one building block of the momentum operator `reps` times on the handle's
 * stream and return without synchronising, so that a caller can time it with events
 * recorded on that stream.  Operands are the handle's own work buffers (their
 * contents are whatever the last computation left; the physical state is not
 * touched).  pass_id: RVE_PASS_* below.  Returns the algorithmic bytes one launch
 * moves through HBM in *bytes_per_launch (may be NULL).  RVE_PASS_CONSTITUTIVE
 * needs the microstructure and evaluates the tangent at the stored strain. */
enum {
  RVE_PASS_FFT_Z = 0,        /* 6-component strided C2C transform along z           */
  RVE_PASS_FFT_Y = 1,        /* 6-component strided C2C transform along y           */
  RVE_PASS_X_TANGENT = 2,    /* row C2R, g K : eps, row R2C on 6 components          */
  RVE_PASS_GRAD = 3,         /* sym(i xi~ (x) u), 3 -> 6 components                  */
  RVE_PASS_DIV = 4,          /* -i xi~ . sigma, 6 -> 3 components                    */
  RVE_PASS_PRECOND = 5,      /* [xi~ . Kbar . xi~]^-1 and <r, z>, 3 components        */
  RVE_PASS_CONSTITUTIVE = 6, /* return map, tangent and reductions                    */
  RVE_PASS_MATVEC = 7,       /* the whole operator application, as the solver runs it:
                                passes 8,1,2,1,9 where available, else 3,0,1,2,1,0,4   */
  RVE_PASS_ZGRAD = 8,        /* CG direction update p = z + beta p, sym(i xi~ (x) p) and
                                the inverse z transform in one pass (even N1 and N3 in
                                16,32,48,64,96,128,256; RVE_E_ARG otherwise)            */
  RVE_PASS_ZDIV = 9,         /* forward z transform, -i xi~ . sigma and block partials
                                of <p, q> in one pass (same grids as RVE_PASS_ZGRAD)    */
  RVE_PASS_PF_ITER = 10      /* the launches of one phase-field CG iteration (eqs. phase,
                                precph: the operator's dot product and updates, the
                                preconditioner's one-component FFT round trip, the
                                convergence test) on the phase-field work vectors        */
};
int rve_diag_pass(struct rve_s* h, int32_t pass_id, int32_t reps, double* bytes_per_launch);

/* Live timing of one operator kernel inside the solver's own CG iterations: while on
 * (on > 0), the launch of the row tangent pass (pass_id RVE_PASS_X_TANGENT; other ids:
 * RVE_E_ARG) in every on-th CG iteration (k = 0, on, 2 on, ... of each solve; on = 1:
 * every iteration) records its start and end into a HIP event pair (hipExtLaunchKernel on
 * the handle's stream); those iterations are launched eagerly instead of replayed from
 * graphs (the event-recording launch costs the kernels around it a few microseconds, which
 * a sparse sample keeps out of most iterations).  on = 0 switches timing off; on < 0:
 * RVE_E_ARG.  Launches that follow convergence within a batch (which return at once) are
 * not counted.  rve_diag_pass_time returns the number of timed launches and their summed
 * duration [ms] since its previous call, and resets both. */
int rve_diag_time_pass(struct rve_s* h, int32_t pass_id, int32_t on);
int rve_diag_pass_time(struct rve_s* h, int64_t* launches, double* total_ms);

/* ---- serving: many independent solves at once -------------------------------------
 * Advance n independent handles by one load increment each, concurrently: one host
 * thread drives each handle (every handle was created on its own stream), so the
 * kernels of the n increments overlap on the device.  This is the tick of a
 * continuous-batching server: a caller admits new handles and retires finished ones
 * between ticks.  deps: n x 6 macroscopic strain increments; dt: n time steps;
 * status: n per-handle return codes (as rve_step_increment); stats: n reports or NULL.
 * Each handle's results are bitwise those of stepping it alone.  Returns RVE_OK when
 * every handle succeeded, otherwise the first failing handle's code.  The handles must
 * be distinct; the call returns after all increments have finished. */
int rve_pool_step(struct rve_s* const* handles, int32_t n, const double* deps, const double* dt,
                  int32_t* status, rve_stats* stats);

/* Serving pool: many handles in one device arena owned by the caller (kept alive until
 * rve_pool_destroy), for servers that admit and retire solves continuously without a
 * device allocation per request.  A handle created in the pool takes its footprint
 * (rve_footprint_bytes, rounded up to 256 bytes) from the first free range of the arena
 * that holds it, and rve_destroy returns the range; neighbouring free ranges merge.
 * Admission by memory is the create call: RVE_E_NOMEM when no free range fits (the
 * message gives the size and the largest free range).  Pool calls are thread-safe; the
 * handles are used as any handle (one thread at a time each) and may be stepped together
 * with rve_pool_step. */
struct rve_pool_s;
/* dev_arena of arena_bytes bytes (aligned up to 256 bytes here).  Errors: RVE_E_ARG (null
 * arena or output, or less than 256 usable bytes). */
int rve_pool_create(void* dev_arena, size_t arena_bytes, struct rve_pool_s** out);
/* As rve_create, with the arena range taken from the pool.  Errors: those of rve_create,
 * RVE_E_NOMEM (no free range fits). */
int rve_create_in_pool(struct rve_pool_s* pool, const rve_desc* d, void* hip_stream,
                       struct rve_s** out);
/* Free bytes of the pool, and in *largest_range (if not NULL) its largest free range. */
size_t rve_pool_free_bytes(struct rve_pool_s* pool, size_t* largest_range);
/* Releases the pool (not the arena).  Errors: RVE_E_STATE while handles of it are alive. */
int rve_pool_destroy(struct rve_pool_s* pool);

typedef struct rve_s* rve_t;

#ifdef __cplusplus
}
#endif

#endif /* RVE_H */
