// Host driver and C ABI: arena layout, crystal tables, Algorithm 1 with the Newton /
// Krylov momentum solver, the phase-field solver, the history commit and the GND
// update.  Every kernel runs on the handle's stream; the host only reads scalars.
#include "../../include/rve.h"
#include "kernels.h"

#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <new>
#include <condition_variable>
#include <mutex>
#include <string>
#include <thread>
#include <type_traits>
#include <vector>

using namespace rvefft;

namespace {

thread_local std::string g_err;
const bool g_debug = std::getenv("RVE_DEBUG") != nullptr;
// RVE_POOL_BATCH=0 (read at every rve_pool_step): every handle's CG solve runs on its own
// (for comparisons)
// Where the convergence test of a CG iteration runs: in its own single-block kernel before
// the next inverse z pass (default), or inside every block of that pass (RVE_CG_CHECK=inline,
// where each block first sums the step's partials: at one resident block per CU that
// latency is exposed once per block)
bool cg_check_inline_mode() {
  static const bool v = [] {
    const char* e = std::getenv("RVE_CG_CHECK");
    return e && std::strcmp(e, "inline") == 0;
  }();
  return v;
}

bool pool_batching_off() {
  const char* e = std::getenv("RVE_POOL_BATCH");
  return e && e[0] == '0';
}

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                   \
  do {                                                                                 \
    hipError_t e_ = (expr);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail(RVE_E_DEVICE, std::string(#expr) + ": " + hipGetErrorString(e_));    \
  } while (0)

bool smooth23(int n) {
  if (n < 1 || n > kMaxN) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

double now_ms() {
  return std::chrono::duration<double, std::milli>(
             std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---- crystal tables (host, FP64) ---------------------------------------------------
// The 12 FCC slip systems: plane normals {111} with three <110> directions each.
const double kSlipN[12][3] = {{1, 1, 1},  {1, 1, 1},  {1, 1, 1},  {-1, 1, 1}, {-1, 1, 1}, {-1, 1, 1},
                              {1, -1, 1}, {1, -1, 1}, {1, -1, 1}, {1, 1, -1}, {1, 1, -1}, {1, 1, -1}};
const double kSlipS[12][3] = {{0, 1, -1}, {1, 0, -1}, {1, -1, 0}, {0, 1, -1}, {1, 0, 1}, {1, 1, 0},
                              {0, 1, 1},  {1, 0, -1}, {1, 1, 0},  {0, 1, 1},  {1, 0, 1}, {1, -1, 0}};
// The 6 <110> screw line directions.
const double kScrew[6][3] = {{1, 1, 0}, {1, -1, 0}, {1, 0, 1}, {1, 0, -1}, {0, 1, 1}, {0, 1, -1}};

const int kPairs[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};

void normalize3(double v[3]) {
  const double s = std::sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
  for (int i = 0; i < 3; ++i) v[i] /= s;
}

void quat_rot(const double* q, double R[3][3]) {
  double w = q[0], x = q[1], y = q[2], z = q[3];
  const double s = std::sqrt(w * w + x * x + y * y + z * z);
  w /= s; x /= s; y /= s; z /= s;
  R[0][0] = 1 - 2 * (y * y + z * z); R[0][1] = 2 * (x * y - w * z); R[0][2] = 2 * (x * z + w * y);
  R[1][0] = 2 * (x * y + w * z); R[1][1] = 1 - 2 * (x * x + z * z); R[1][2] = 2 * (y * z - w * x);
  R[2][0] = 2 * (x * z - w * y); R[2][1] = 2 * (y * z + w * x); R[2][2] = 1 - 2 * (x * x + y * y);
}

// Gauss-Jordan inverse with partial pivoting of an n x n row-major matrix.
bool invert(std::vector<double>& A, int n) {
  std::vector<double> I(n * n, 0.0);
  for (int i = 0; i < n; ++i) I[i * n + i] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(I[c * n + k], I[piv * n + k]);
    }
    const double d = A[c * n + c];
    for (int k = 0; k < n; ++k) { A[c * n + k] /= d; I[c * n + k] /= d; }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      const double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) { A[r * n + k] -= f * A[c * n + k]; I[r * n + k] -= f * I[c * n + k]; }
    }
  }
  A = I;
  return true;
}

// One grain's table: rotated Mandel stiffness and compliance, Mandel Schmid tensors,
// s (x) n and the rotation.
bool grain_table(const double* q, double C11, double C12, double C44, double* out) {
  double R[3][3];
  quat_rot(q, R);
  double c0[3][3][3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j)
      for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l) {
          double v = C12 * (i == j) * (k == l) + C44 * ((i == k) * (j == l) + (i == l) * (j == k));
          if (i == j && j == k && k == l) v += C11 - C12 - 2.0 * C44;
          c0[i][j][k][l] = v;
        }
  // rotate each index: C'_ijkl = R_ia R_jb R_kc R_ld C_abcd, in four contractions
  double t1[3][3][3][3], t2[3][3][3][3];
  auto contract = [&](double (&src)[3][3][3][3], double (&dst)[3][3][3][3], int slot) {
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        for (int k = 0; k < 3; ++k)
          for (int l = 0; l < 3; ++l) {
            double s = 0.0;
            for (int a = 0; a < 3; ++a) {
              const int idx[4] = {i, j, k, l};
              int src_idx[4] = {i, j, k, l};
              src_idx[slot] = a;
              s += R[idx[slot]][a] * src[src_idx[0]][src_idx[1]][src_idx[2]][src_idx[3]];
            }
            dst[i][j][k][l] = s;
          }
  };
  contract(c0, t1, 0);
  contract(t1, t2, 1);
  contract(t2, t1, 2);
  contract(t1, t2, 3);
  const double w[6] = {1, 1, 1, std::sqrt(2.0), std::sqrt(2.0), std::sqrt(2.0)};
  std::vector<double> Cm(36);
  for (int a = 0; a < 6; ++a)
    for (int b = 0; b < 6; ++b)
      Cm[a * 6 + b] = w[a] * w[b] * t2[kPairs[a][0]][kPairs[a][1]][kPairs[b][0]][kPairs[b][1]];
  std::vector<double> Sm = Cm;
  if (!invert(Sm, 6)) return false;
  for (int i = 0; i < 36; ++i) { out[GT_C + i] = Cm[i]; out[GT_S + i] = Sm[i]; }
  for (int a = 0; a < 12; ++a) {
    double s0[3] = {kSlipS[a][0], kSlipS[a][1], kSlipS[a][2]};
    double n0[3] = {kSlipN[a][0], kSlipN[a][1], kSlipN[a][2]};
    normalize3(s0);
    normalize3(n0);
    double s[3], n[3];
    for (int i = 0; i < 3; ++i) {
      s[i] = R[i][0] * s0[0] + R[i][1] * s0[1] + R[i][2] * s0[2];
      n[i] = R[i][0] * n0[0] + R[i][1] * n0[1] + R[i][2] * n0[2];
    }
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) out[GT_SN + a * 9 + i * 3 + j] = s[i] * n[j];
    for (int b = 0; b < 6; ++b) {
      const int i = kPairs[b][0], j = kPairs[b][1];
      out[GT_P + a * 6 + b] = w[b] * 0.5 * (s[i] * n[j] + s[j] * n[i]);
    }
  }
  for (int i = 0; i < 9; ++i) out[GT_R + i] = R[i / 3][i % 3];
  return true;
}

// Crystal-frame constants shared by all grains.
void crystal_frame(double C11, double C12, double C44, CrystalFrame* cf) {
  const double w[6] = {1, 1, 1, std::sqrt(2.0), std::sqrt(2.0), std::sqrt(2.0)};
  for (int a = 0; a < 12; ++a) {
    double s[3] = {kSlipS[a][0], kSlipS[a][1], kSlipS[a][2]};
    double n[3] = {kSlipN[a][0], kSlipN[a][1], kSlipN[a][2]};
    normalize3(s);
    normalize3(n);
    for (int b = 0; b < 6; ++b) {
      const int i = kPairs[b][0], j = kPairs[b][1];
      cf->P[a * 6 + b] = w[b] * 0.5 * (s[i] * n[j] + s[j] * n[i]);
    }
  }
  cf->c11 = C11;
  cf->c12 = C12;
  cf->c66 = 2.0 * C44;
  const double det = (C11 - C12) * (C11 + 2.0 * C12);
  cf->s11 = (C11 + C12) / det;
  cf->s12 = -C12 / det;
  cf->s66 = 1.0 / (2.0 * C44);
}

// Crystal-frame unit slip directions and plane normals with the cubic Mandel constants
// (finite-strain return map).
void fs_frame(double C11, double C12, double C44, FsFrame* ff) {
  CrystalFrame cf;
  crystal_frame(C11, C12, C44, &cf);
  for (int a = 0; a < 12; ++a) {
    double s[3] = {kSlipS[a][0], kSlipS[a][1], kSlipS[a][2]};
    double n[3] = {kSlipN[a][0], kSlipN[a][1], kSlipN[a][2]};
    normalize3(s);
    normalize3(n);
    for (int i = 0; i < 3; ++i) {
      ff->s[3 * a + i] = s[i];
      ff->n[3 * a + i] = n[i];
    }
  }
  ff->c11 = cf.c11; ff->c12 = cf.c12; ff->c66 = cf.c66;
  ff->s11 = cf.s11; ff->s12 = cf.s12; ff->s66 = cf.s66;
}

// Q = (A A^T)^-1 for the 9 x 18 crystal-frame GND basis (12 edge: s (x) (s x n),
// 6 screw: d (x) d), row-major vec.
bool gnd_q(double* Q) {
  std::vector<double> A(9 * 18, 0.0);
  for (int a = 0; a < 12; ++a) {
    double s[3] = {kSlipS[a][0], kSlipS[a][1], kSlipS[a][2]};
    double n[3] = {kSlipN[a][0], kSlipN[a][1], kSlipN[a][2]};
    normalize3(s);
    normalize3(n);
    const double t[3] = {s[1] * n[2] - s[2] * n[1], s[2] * n[0] - s[0] * n[2], s[0] * n[1] - s[1] * n[0]};
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[(i * 3 + j) * 18 + a] = s[i] * t[j];
  }
  for (int b = 0; b < 6; ++b) {
    double d[3] = {kScrew[b][0], kScrew[b][1], kScrew[b][2]};
    normalize3(d);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) A[(i * 3 + j) * 18 + 12 + b] = d[i] * d[j];
  }
  std::vector<double> M(81, 0.0);
  for (int i = 0; i < 9; ++i)
    for (int j = 0; j < 9; ++j) {
      double s = 0.0;
      for (int k = 0; k < 18; ++k) s += A[i * 18 + k] * A[j * 18 + k];
      M[i * 9 + j] = s;
    }
  if (!invert(M, 9)) return false;
  for (int i = 0; i < 81; ++i) Q[i] = M[i];
  return true;
}

}  // namespace

// ---- handle ------------------------------------------------------------------------
// Same-size handles of one rve_pool_step tick whose CG solves run as batched launches.
struct CgJob {
  rve_s* h = nullptr;
  int iters = 0;
  int rc = 0;
  std::string msg;
  bool done = false;
};
struct CgGroup {
  std::mutex mu;
  std::condition_variable cv;
  std::vector<CgJob*> pending;
  bool leader = false;
  int members = 0;          // handles of the group still inside their increment
  int wait_us = 400;        // a leader's wait for the other members to reach their CG solve
};

struct rve_s {
  rve_desc d;
  Grid g;
  Plans pl;
  hipStream_t st;
  bool f64;               // spectral precision
  char* base = nullptr;
  size_t cap = 0, used = 0;
  // state (FP64)
  double *eps, *eps_t, *eps_prev, *deps, *sig, *sig_t, *epsp, *beta, *gslip, *rho_ssd, *rho_gnd,
      *wp, *gs, *H, *wcrit, *trig, *phi, *phi_t, *phi_prev, *S, *wep, *gw;
  int* grain;
  double* gtab;
  CrystalFrame cf;        // crystal-frame slip and elasticity constants
  double* Q81;
  void* gK;               // 21 N reals (R)
  void* spec;             // 9 NH complex (R): operator work and GND scratch
  void* cg[6];            // x, r, z, p, q, b : 3 NH complex each
  void* gm_basis = nullptr;  // GMRES option: m + 1 basis vectors of 3 NH complex
  double* rbuf;           // 9 N doubles: phase-field vectors / Nye tensor / stress readback
  double* partial;        // reduction partials
  double* scal;           // device scalars
  int* failc;
  // HIP graphs of one CG iteration of each parity (captured at first use; the
  // launches of an iteration depend on the handle and the parity only)
  bool use_graphs = true;
  hipGraphExec_t cg_exec[2] = {nullptr, nullptr};
  int graph_mask = 0;     // stress-control mask the captured graphs were built for
  // live timing of the row (x) tangent pass inside the CG iterations (rve_diag_time_pass):
  // an event pair around the launch of every time_xt-th iteration (0: off), harvested
  // after each batch; launches of a batch after convergence (no-ops) are not counted
  int time_xt = 0;
  std::vector<hipEvent_t> xt_ev;          // 2 per launch of the current batch
  std::vector<int> xt_iter;               // CG iteration of each pair
  int xt_used = 0;
  long long xt_launches = 0;
  double xt_ms = 0.0;
  // macro stress and strain at time t (tensor components), the reference of the next
  // increment's stress-controlled components
  double msig_t[6] = {0, 0, 0, 0, 0, 0}, meps_t[6] = {0, 0, 0, 0, 0, 0};
  double* hs = nullptr;   // pinned host scalars
  bool micro = false;
  int static_dev = -1;    // >= 0: the arena is that device's static scratch array
  struct rve_pool_s* pool = nullptr;   // the serving pool whose arena holds this one's
  size_t pool_off = 0, pool_len = 0;
  double hs_static[544];  // host scalars of a static-arena handle (no pinned allocation)
  // finite-strain kinematics (rve_desc.kinematics == RVE_KIN_FINITE): deformation gradient
  // at t + dt, at t and at the previous alternating pass, the Newton correction, the
  // effective first Piola-Kirchhoff stress, the plastic deformation and its trial value
  // (9 each, row-major), and the per-voxel increments (sum tau dgamma, sum |dgamma|,
  // dLp : dLp, W_e+); the tangent field then holds 81 FP64 entries per voxel and sig the
  // crystal-frame second Piola-Kirchhoff stress (the return map's warm start)
  // serving: the handle's group of same-size handles inside rve_pool_step (their CG
  // iterations advance in shared launches), its events and the slot-offset table (in the
  // arena) of a batch it leads
  CgGroup* cg_group = nullptr;
  int batch_peak = 1;     // largest batch this handle's CG solves ran in (this increment)
  hipEvent_t cg_ready = nullptr, cg_done = nullptr;
  long long* slotd = nullptr;
  // GND-coupled hardening option: the strength at t_n, the next pass's strength and the
  // end-of-increment SSD and GND densities of the current pass
  double *g_n = nullptr, *g_next = nullptr, *rho_ssd_tr = nullptr, *rho_gnd_tr = nullptr,
         *g_res = nullptr;
  // plane-stress option: the condensed effective stress of the in-plane balance (6 N) and
  // the per-voxel recovery of the out-of-plane strain correction, B and r (12 N)
  double *ps_sig = nullptr, *ps_rec = nullptr;
  bool fs = false;
  double *fs_F = nullptr, *fs_Ft = nullptr, *fs_Fprev = nullptr, *fs_dF = nullptr,
         *fs_P = nullptr, *fs_Fp = nullptr, *fs_fptr = nullptr, *fs_aux = nullptr;
  FsFrame ff;
  long long n_preset = 0; // voxels of the pre-set crack (phi0 = 1)
  int n_grains = 0;
  int device = 0;         // device current at creation
};

namespace {

enum { SC_K = 0,        // 28 constitutive sums (21 gK, g w, 6 g sigma)
       SC_KBAR = 32,    // 21 mean tangent
       SC_RZ0 = 56, SC_RZ1 = 57, SC_PQ = 58, SC_RR = 59, SC_BB = 60,
       SC_FLAG = 61, SC_ITER = 62, SC_TOL2 = 63,
       SC_ZERO = 80, SC_ONE = 81, SC_RRN = 82, SC_RZN = 83,
       SC_MISC = 64,    // generic reduce outputs (16)
       SC_M0 = 360,     // 72: macro-block preconditioner and the block it inverts (mixed control)
       SC_DE = 132,     // 6: macro strain increment of a Newton step (mixed control)
       SC_GN = 140,     // GMRES: a norm
       SC_GM = 144,     // GMRES: Gram-Schmidt coefficients, first pass (up to 65)
       SC_GM2 = 216,    // GMRES: second pass
       SC_GY = 288,     // GMRES: least-squares solution (up to 64)
       SC_FK = 432,     // finite strain: 81 mean tangent
       SC_FM = 520,     // finite strain: 21 commit reductions
       SC_N = 544 };

size_t align_up(size_t x) { return (x + 255) & ~(size_t)255; }

// Reduction buffer: the divergence pass's partials from 0, the CG step's from
// cg_partial_offset() (at most 2 x kCgMaxBlocks: every block of the next inverse z pass sums
// them).  The CG step's blocks write their partials while other blocks of the same launch
// still sum the divergence pass's, so the two ranges must not overlap: the fused divergence
// pass launches (N1/2/T) N2 3 blocks with tiles of T >= 8 bins (plus one partial of the macro
// stress), at most 3 N1 N2 / 16 + 1.
constexpr long long kCgPartialMin = (long long)kMaxRedBlocks * 16;
constexpr int kMaxBatch = 64;         // RVEs of one batched CG launch
constexpr int kCgMaxBlocks = 1024;   // 512 measured 4 us slower per FP32 iteration at 128^3

long long max_div_partials(const Grid& g) {
  const long long fused = 3LL * g.n1 * g.n2 / 16 + 1;
  return fused > kMaxRedBlocks + 1 ? fused : kMaxRedBlocks + 1;
}
long long cg_partial_offset(const Grid& g) {
  const long long need = (max_div_partials(g) + 63) / 64 * 64;
  return need > kCgPartialMin ? need : kCgPartialMin;
}
// (also the return map's per-block constitutive sums: RED_CONST per 256-voxel block)
long long partial_count(const Grid& g) {
  const long long base = cg_partial_offset(g) + kMaxRedBlocks * 16;
  const long long sums = (long long)RED_CONST * ((g.nvox + 255) / 256);
  return base > sums ? base : sums;
}



// Bump allocation of every buffer; with h->base == nullptr only the size is summed.
void layout(rve_s* h) {
  const long long N = h->g.nvox, NH = h->g.nspec;
  const size_t csz = h->f64 ? 16 : 8, rsz = h->f64 ? 8 : 4;
  h->used = 0;
  auto take = [&](size_t bytes) -> void* {
    void* p = h->base ? (void*)(h->base + h->used) : nullptr;
    h->used += align_up(bytes);
    return p;
  };
  auto fd = [&](long long cnt) { return (double*)take((size_t)cnt * 8); };
  h->eps = fd(6 * N); h->eps_t = fd(6 * N); h->eps_prev = fd(6 * N); h->deps = fd(6 * N);
  h->sig = fd(6 * N); h->sig_t = fd(6 * N); h->epsp = fd(6 * N); h->beta = fd(9 * N);
  h->gslip = fd(N); h->rho_ssd = fd(N); h->rho_gnd = fd(N); h->wp = fd(N); h->gs = fd(N);
  h->H = fd(N); h->wcrit = fd(N); h->trig = fd(N); h->phi = fd(N); h->phi_t = fd(N);
  h->phi_prev = fd(N); h->S = fd(N); h->wep = fd(N); h->gw = fd(N);
  h->grain = (int*)take((size_t)N * 4);
  h->gtab = fd((long long)h->d.max_grains * GT_STRIDE);
  h->Q81 = fd(81);
  h->gK = take((size_t)(h->fs ? 81 * 8 : 21 * rsz) * N);
  h->spec = take((size_t)9 * NH * csz);
  for (int i = 0; i < 6; ++i) h->cg[i] = take((size_t)3 * NH * csz);
  h->gm_basis = h->d.krylov == RVE_KRYLOV_GMRES
                    ? take((size_t)(h->d.gmres_restart + 1) * 3 * NH * csz)
                    : nullptr;
  h->rbuf = fd(9 * N);
  h->partial = fd(partial_count(h->g));
  if (h->d.gnd_coupling) {
    h->g_n = fd(N); h->g_next = fd(N); h->rho_ssd_tr = fd(N); h->rho_gnd_tr = fd(N);
    h->g_res = fd(N);
  }
  if (h->d.plane_stress) {
    h->ps_sig = fd(6 * N); h->ps_rec = fd(12 * N);
  }
  if (h->fs) {
    h->fs_F = fd(9 * N); h->fs_Ft = fd(9 * N); h->fs_Fprev = fd(9 * N); h->fs_dF = fd(9 * N);
    h->fs_P = fd(9 * N); h->fs_Fp = fd(9 * N); h->fs_fptr = fd(9 * N); h->fs_aux = fd(4 * N);
  }
  h->scal = fd(SC_N);
  h->slotd = (long long*)take(kMaxBatch * 8);
  h->failc = (int*)take(256);
  for (int a = 0; a < 3; ++a) {
    h->pl.tw64[a] = take((size_t)h->pl.ax[a].n * 16);
    h->pl.tw32[a] = take((size_t)h->pl.ax[a].n * 8);
  }
}

int validate(const rve_desc* d) {
  if (!d) return fail(RVE_E_ARG, "null description");
  for (int a = 0; a < 3; ++a)
    if (!smooth23(d->n[a])) return fail(RVE_E_ARG, "grid sizes must be 2^p 3^q in [1, 512]");
  if (d->precision != RVE_FP64 && d->precision != RVE_MIXED)
    return fail(RVE_E_ARG, "precision must be RVE_FP64 or RVE_MIXED");
  const double pos[] = {d->h, d->C44, d->tau_c0, d->rho0, d->burgers, d->ell,
                        d->Gc, d->k_res, d->tol_stag, d->tol_newton, d->tol_lin};
  for (double v : pos)
    if (!(v > 0.0) || !std::isfinite(v)) return fail(RVE_E_ARG, "non-positive or non-finite constant");
  if (d->krylov != RVE_KRYLOV_CG && d->krylov != RVE_KRYLOV_GMRES)
    return fail(RVE_E_ARG, "krylov must be RVE_KRYLOV_CG or RVE_KRYLOV_GMRES");
  if (d->krylov == RVE_KRYLOV_GMRES && (d->gmres_restart < 1 || d->gmres_restart > 64))
    return fail(RVE_E_ARG, "gmres_restart must be in 1..64");
  if (d->deriv != RVE_DERIV_SPECTRAL && d->deriv != RVE_DERIV_ROTATED)
    return fail(RVE_E_ARG, "deriv must be RVE_DERIV_SPECTRAL or RVE_DERIV_ROTATED");
  if (d->pf_dirichlet != 0 && d->pf_dirichlet != 1) return fail(RVE_E_ARG, "pf_dirichlet must be 0 or 1");
  if (d->gnd_coupling != 0 && d->gnd_coupling != 1)
    return fail(RVE_E_ARG, "gnd_coupling must be 0 or 1");
  if (d->gnd_coupling && (d->material != RVE_MAT_DUNNE || d->kinematics != RVE_KIN_SMALL))
    return fail(RVE_E_ARG, "gnd_coupling needs the Taylor hardening of RVE_MAT_DUNNE and "
                           "small-strain kinematics");
  if (d->plane_stress != 0 && d->plane_stress != 1)
    return fail(RVE_E_ARG, "plane_stress must be 0 or 1");
  if (d->plane_stress && (d->n[2] != 1 || d->kinematics != RVE_KIN_SMALL))
    return fail(RVE_E_ARG, "plane_stress needs a grid one voxel thick (n[2] = 1) and "
                           "small-strain kinematics");
  if (d->kinematics != RVE_KIN_SMALL && d->kinematics != RVE_KIN_FINITE)
    return fail(RVE_E_ARG, "kinematics must be RVE_KIN_SMALL or RVE_KIN_FINITE");
  if (d->kinematics == RVE_KIN_FINITE &&
      (d->precision != RVE_FP64 || d->krylov != RVE_KRYLOV_GMRES || d->deriv != RVE_DERIV_SPECTRAL))
    return fail(RVE_E_ARG, "finite-strain kinematics run in FP64 with the GMRES solver and the "
                           "spectral derivative");
  if (d->material != RVE_MAT_POWER && d->material != RVE_MAT_DUNNE)
    return fail(RVE_E_ARG, "material must be RVE_MAT_POWER or RVE_MAT_DUNNE");
  if (d->material == RVE_MAT_POWER) {
    if (!(d->gdot0 > 0.0) || !std::isfinite(d->gdot0) || !(d->n_exp > 0.0) ||
        !std::isfinite(d->n_exp))
      return fail(RVE_E_ARG, "non-positive or non-finite power-law constant");
  } else {
    const double th[] = {d->rho_m, d->v_D, d->dF, d->k_B, d->T, d->dV, d->mu};
    for (double v : th)
      if (!(v > 0.0) || !std::isfinite(v))
        return fail(RVE_E_ARG, "non-positive or non-finite constant of the thermally activated rule");
    const double kT = d->k_B * d->T;
    const double A = d->rho_m * d->burgers * d->burgers * d->v_D * std::exp(-d->dF / kT);
    if (!(A > 0.0) || !std::isfinite(A) || !std::isfinite(d->dV / kT))
      return fail(RVE_E_ARG, "rate prefactor of the thermally activated rule out of range");
  }
  const double nonneg[] = {d->h_lin, d->lambda_ssd, d->xi_store, d->G_crit, d->ell_fp};
  for (double v : nonneg)
    if (!(v >= 0.0) || !std::isfinite(v)) return fail(RVE_E_ARG, "negative or non-finite constant");
  if (!(d->C11 > d->C12) || !(d->C11 + 2 * d->C12 > 0))
    return fail(RVE_E_ARG, "elastic constants are not positive definite");
  if (d->max_stag < 1 || d->max_newton < 1 || d->max_krylov < 1 || d->max_grains < 1)
    return fail(RVE_E_ARG, "iteration limits and max_grains must be >= 1");
  return RVE_OK;
}

void init_grid(rve_s* h) {
  Grid& g = h->g;
  g.n1 = h->d.n[0]; g.n2 = h->d.n[1]; g.n3 = h->d.n[2];
  g.n1h = g.n1 / 2 + 1;
  g.nvox = (long long)g.n1 * g.n2 * g.n3;
  g.nspec = (long long)g.n1h * g.n2 * g.n3;
  g.h = h->d.h;
  g.L1 = g.n1 * g.h; g.L2 = g.n2 * g.h; g.L3 = g.n3 * g.h;
  g.sch = h->d.deriv;
  h->pl.g = g;
  for (int a = 0; a < 3; ++a) make_axis_plan(h->d.n[a], &h->pl.ax[a]);
  h->f64 = (h->d.precision == RVE_FP64);
  h->fs = (h->d.kinematics == RVE_KIN_FINITE);
}

// ---- small helpers on the handle ---------------------------------------------------
struct Ctx {
  rve_s* h;
  hipStream_t st;
  long long N, NH;
};

int sync_read(rve_s* h, int first, int count) {
  HIPCHK(hipMemcpyAsync(h->hs + first, h->scal + first, count * sizeof(double),
                        hipMemcpyDeviceToHost, h->st));
  HIPCHK(hipStreamSynchronize(h->st));
  HIPCHK(hipGetLastError());
  return RVE_OK;
}

template <typename R>
struct Ops {
  typedef cplx<R> C;
  rve_s* h;
  hipStream_t st;
  long long N, NH;
  C* W;            // 6-component operator work (first 6 comps of spec)
  C* v(int i) { return (C*)h->cg[i]; }
  R* gK() { return (R*)h->gK; }

  // mixed macroscopic control: stress-controlled components (bit c for xx yy zz yz xz
  // xy; 0 = strain control) and the scale s of the macro unknowns in the zero bin
  int mask = 0;
  double s_mac = 0.0;
  const double* m0() const { return mask ? h->scal + SC_M0 : nullptr; }

  explicit Ops(rve_s* hh) : h(hh), st(hh->st), N(hh->g.nvox), NH(hh->g.nspec) { W = (C*)h->spec; }

  // finite-strain operator (the handle's kinematics): 9-component gradient and
  // divergence, 81-entry tangent applied in real space, preconditioner from the 81-entry
  // mean tangent (FP64 only)
  bool fs = false;
  void precond(const C* r, C* z) {
    if constexpr (std::is_same_v<R, double>) {
      if (fs) {
        launch_fs_precond(h->pl, r, z, NH, h->scal + SC_FK, st);
        return;
      }
    }
    launch_precond<R>(h->pl, r, z, NH, h->scal + SC_KBAR, h->partial, st, nullptr, m0());
  }
  // q = -i xi~_j F{ gK_ijkl F^-1{ i xi~_l p_k } } (eqs. fdef, newton)
  void matvec_fs(const C* p, C* q, const double* stop) {
    if constexpr (std::is_same_v<R, double>) {
      launch_fs_grad(h->pl, p, NH, W, NH, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 9, 2, true, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 9, 1, true, st, stop);
      launch_x_c2r<R>(h->pl, W, NH, h->rbuf, true, N, 9, 1.0 / (double)N, 0, st, stop);
      launch_fs_tangent(h->rbuf, N, (const double*)h->gK, st, stop);
      launch_x_r2c<R>(h->pl, h->rbuf, true, N, nullptr, 0.0, W, NH, 9, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 9, 1, false, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 9, 2, false, st, stop);
      launch_fs_div(h->pl, W, NH, q, NH, -1.0, st, stop);
    }
  }

  // forward 3-D real FFT of ncomp real comps (stride in_cs) into spec comps
  void fwd(const void* in, bool in64, long long in_cs, int ncomp, C* out, const double* phi = nullptr) {
    launch_x_r2c<R>(h->pl, in, in64, in_cs, phi, h->d.k_res, out, NH, ncomp, st);
    launch_fft_yz<R>(h->pl, out, NH, ncomp, 1, false, st);
    launch_fft_yz<R>(h->pl, out, NH, ncomp, 2, false, st);
  }
  // inverse 3-D FFT (in place on spec comps, then rows to real out)
  void inv(C* in, int ncomp, void* out, bool out64, long long out_cs, double scale, int acc) {
    launch_fft_yz<R>(h->pl, in, NH, ncomp, 2, true, st);
    launch_fft_yz<R>(h->pl, in, NH, ncomp, 1, true, st);
    launch_x_c2r<R>(h->pl, in, NH, out, out64, out_cs, ncomp, scale, acc, st);
  }
  // q = B p = - i xi~ . F{ gK : F^-1{ sym(i xi~ (x) p) } }; every launch is skipped
  // once *stop is non-zero (device-side Krylov termination).
  // With the fused z passes, `scratch` (3 NH) receives the copy of p the inverse pass
  // stores as the updated direction, and the partials of <p, q> are left unused.
  void matvec(const C* p, C* q, C* scratch, const double* stop = nullptr) {
    if (fs) {
      matvec_fs(p, q, stop);
      return;
    }
    // (mixed control: the stress-controlled macro strains in the zero bin of p enter the
    // strain, and q(0) takes the macro stress, as in the CG iterations)
    const bool fz = fused_z_available<R>(h->pl);
    const long long zst = (long long)h->g.n1h * h->g.n2;
    if (fz) {
      launch_zgrad_inv<R>(h->pl, p, p, scratch, NH, h->scal, SC_ZERO, SC_ONE, W, st, stop);
      if (mask)
        launch_macro_strain<R>(W, NH, p, NH, s_mac, 0.0, mask, h->g.n3, zst, nullptr, st, stop);
    } else {
      launch_sym_grad<R>(h->pl, p, NH, W, NH, st, stop);
      if (mask) launch_macro_strain<R>(W, NH, p, NH, s_mac, 0.0, mask, 1, 0, nullptr, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 6, 2, true, st, stop);
    }
    launch_fft_yz<R>(h->pl, W, NH, 6, 1, true, st, stop);
    launch_x_tangent<R>(h->pl, W, NH, gK(), 1.0 / (double)N, st, stop);
    launch_fft_yz<R>(h->pl, W, NH, 6, 1, false, st, stop);
    if (fz) {
      const int nbd = launch_zdiv_fwd<R>(h->pl, W, q, p, NH, h->partial, st, stop);
      if (mask)
        launch_macro_stress<R>(W, NH, q, p, NH, s_mac, mask, h->g.n3, zst, h->partial + nbd, st,
                               stop);
    } else {
      launch_fft_yz<R>(h->pl, W, NH, 6, 2, false, st, stop);
      launch_div<R>(h->pl, W, NH, q, NH, -1.0, st, stop);
      if (mask) launch_macro_stress<R>(W, NH, q, p, NH, s_mac, mask, 1, 0, h->partial, st, stop);
    }
  }
  // The row tangent pass of CG iteration k, timing itself into an event pair while live
  // timing is on.
  bool timed_iter(int k) const { return h->time_xt > 0 && k % h->time_xt == 0; }
  void timed_x_tangent(int k, const double* stop) {
    if (!timed_iter(k)) {
      launch_x_tangent<R>(h->pl, W, NH, gK(), 1.0 / (double)N, st, stop);
      return;
    }
    if ((int)h->xt_ev.size() < 2 * (h->xt_used + 1)) {
      hipEvent_t a = nullptr, b = nullptr;
      if (hipEventCreate(&a) == hipSuccess) h->xt_ev.push_back(a);
      if (hipEventCreate(&b) == hipSuccess) h->xt_ev.push_back(b);
      h->xt_iter.resize(h->xt_ev.size() / 2);
    }
    const bool ok = (int)h->xt_ev.size() >= 2 * (h->xt_used + 1);
    if (!ok) {
      launch_x_tangent<R>(h->pl, W, NH, gK(), 1.0 / (double)N, st, stop);
      return;
    }
    // the launch timestamps its own start and end into the pair
    launch_x_tangent<R>(h->pl, W, NH, gK(), 1.0 / (double)N, st, stop, h->xt_ev[2 * h->xt_used],
                        h->xt_ev[2 * h->xt_used + 1]);
    h->xt_iter[h->xt_used++] = k;
  }
  // After a batch (stream synchronised): add the pairs of the iterations that ran.
  int harvest_x_tangent(int iters_run) {
    for (int i = 0; i < h->xt_used; ++i) {
      if (h->xt_iter[i] >= iters_run) continue;
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, h->xt_ev[2 * i], h->xt_ev[2 * i + 1]));
      h->xt_ms += ms;
      ++h->xt_launches;
    }
    h->xt_used = 0;
    return RVE_OK;
  }

  // Restarted GMRES(m) on M B du = M c (left preconditioning; the paper's Krylov solver):
  // classical Gram-Schmidt with one re-orthogonalisation, kGmChunk basis vectors per
  // block dot / update launch, Givens rotations and the small least-squares solve on the
  // host; relative tolerance on the preconditioned residual.  Solution in cg[0]; iters
  // counts operator applications.
  int norm(const C* a, double& out) {
    const int nb = launch_sdot<R>(h->pl, a, a, NH, 3, h->partial, st);
    launch_reduce(h->partial, nb, 1, 0, h->scal + SC_GN, st);
    const int rc = sync_read(h, SC_GN, 1);
    out = std::sqrt(h->hs[SC_GN]);
    return rc;
  }
  int gmres(int& iters) {
    const int m = h->d.gmres_restart;
    C *x = v(0), *w = v(1), *t = v(2), *scr = v(3), *b = v(5);
    C* V = (C*)h->gm_basis;
    const long long vs = 3 * NH;
    double* sc = h->scal;
    iters = 0;
    launch_zero(x, (size_t)3 * NH * sizeof(C), st);
    precond(b, V);    // r0 = M c
    double beta;
    int rc;
    if ((rc = norm(V, beta))) return rc;
    if (!(beta > 0.0)) return std::isfinite(beta) ? RVE_OK : fail(RVE_E_NOCONV, "non-finite residual");
    const double tol = h->d.tol_lin * beta;
    std::vector<double> H((size_t)(m + 1) * m, 0.0), cs(m), sn(m), g(m + 1), y(m), hc(m + 1);
    for (;;) {
      launch_caxpby<R>(h->pl, V, 1.0 / beta, nullptr, 0.0, V, NH, st);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      int jl = -1;
      bool conv = false;
      for (int j = 0; j < m; ++j) {
        // w = M P(B V_j), P the Hermitian projection of the self-conjugate planes
        matvec(V + j * vs, t, scr);
        if (!mask) launch_herm_proj<R>(h->pl, t, NH, 3, st);
        precond(t, w);
        for (int pass = 0; pass < 2; ++pass) {
          const int base = pass ? SC_GM2 : SC_GM;
          for (int c0 = 0; c0 <= j; c0 += kGmChunk) {
            const int nv = std::min(kGmChunk, j + 1 - c0);
            const int nb = launch_mdot<R>(h->pl, V + c0 * vs, vs, nv, w, NH, h->partial, st);
            launch_reduce(h->partial, nb, nv, 0, sc + base + c0, st);
          }
          for (int c0 = 0; c0 <= j; c0 += kGmChunk) {
            const int nv = std::min(kGmChunk, j + 1 - c0);
            launch_maxpy<R>(h->pl, V + c0 * vs, vs, nv, sc + base + c0, -1.0, w, NH, st);
          }
        }
        if ((rc = sync_read(h, SC_GM, SC_GM2 - SC_GM + j + 1))) return rc;
        for (int i = 0; i <= j; ++i) hc[i] = h->hs[SC_GM + i] + h->hs[SC_GM2 + i];
        double hn;
        if ((rc = norm(w, hn))) return rc;
        ++iters;
        for (int i = 0; i < j; ++i) {          // previous rotations
          const double a = cs[i] * hc[i] + sn[i] * hc[i + 1];
          hc[i + 1] = -sn[i] * hc[i] + cs[i] * hc[i + 1];
          hc[i] = a;
        }
        const double den = std::hypot(hc[j], hn);
        cs[j] = den > 0.0 ? hc[j] / den : 1.0;
        sn[j] = den > 0.0 ? hn / den : 0.0;
        hc[j] = den;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        for (int i = 0; i <= j; ++i) H[(size_t)i * m + j] = hc[i];
        jl = j;
        if (!std::isfinite(g[j + 1])) return fail(RVE_E_NOCONV, "momentum GMRES breakdown");
        conv = std::fabs(g[j + 1]) <= tol || !(hn > 0.0);
        if (conv || iters >= h->d.max_krylov) break;
        launch_caxpby<R>(h->pl, w, 1.0 / hn, nullptr, 0.0, V + (j + 1) * vs, NH, st);
      }
      // x += V y with H y = g (upper triangular)
      for (int i = jl; i >= 0; --i) {
        double s = g[i];
        for (int k = i + 1; k <= jl; ++k) s -= H[(size_t)i * m + k] * y[k];
        y[i] = s / H[(size_t)i * m + i];
      }
      for (int i = 0; i <= jl; ++i) h->hs[SC_GY + i] = y[i];
      HIPCHK(hipMemcpyAsync(sc + SC_GY, h->hs + SC_GY, (size_t)(jl + 1) * sizeof(double),
                            hipMemcpyHostToDevice, st));
      for (int c0 = 0; c0 <= jl; c0 += kGmChunk) {
        const int nv = std::min(kGmChunk, jl + 1 - c0);
        launch_maxpy<R>(h->pl, V + c0 * vs, vs, nv, sc + SC_GY + c0, 1.0, x, NH, st);
      }
      if (conv) return RVE_OK;
      if (iters >= h->d.max_krylov) return fail(RVE_E_NOCONV, "momentum GMRES reached max_krylov");
      // restart from the preconditioned residual M (c - P B x)
      matvec(x, t, scr);
      if (!mask) launch_herm_proj<R>(h->pl, t, NH, 3, st);
      launch_caxpby<R>(h->pl, b, 1.0, t, -1.0, t, NH, st);
      precond(t, V);
      if ((rc = norm(V, beta))) return rc;
      if (beta <= tol) return RVE_OK;
    }
  }

  // The CG solve of a handle in a pool tick (its set-up done on its own stream): wait at
  // the group's rendezvous; the first waiting thread leads, collects the handles that reach
  // their solve within the group's wait and runs their iterations as batched launches
  // (run_batch); the others sleep until their solve is over.  Every handle's arithmetic is
  // that of its own solve (same kernels and block decomposition, per-handle reductions
  // and convergence flags), so the results do not depend on the company.
  int pcg_batched(int& iters) {
    CgGroup* G = h->cg_group;
    if (!h->cg_ready) HIPCHK(hipEventCreateWithFlags(&h->cg_ready, hipEventDisableTiming));
    HIPCHK(hipEventRecord(h->cg_ready, st));
    CgJob job;
    job.h = h;
    std::unique_lock<std::mutex> lk(G->mu);
    G->pending.push_back(&job);
    G->cv.notify_all();
    while (!job.done) {
      if (!G->leader) {
        G->leader = true;
        const auto t_end =
            std::chrono::steady_clock::now() + std::chrono::microseconds(G->wait_us);
        while ((int)G->pending.size() < G->members && std::chrono::steady_clock::now() < t_end)
          G->cv.wait_until(lk, t_end);
        std::vector<CgJob*> batch;
        batch.swap(G->pending);
        lk.unlock();
        run_batch(batch);
        lk.lock();
        for (CgJob* j : batch) j->done = true;
        G->leader = false;
        G->cv.notify_all();
      } else {
        G->cv.wait(lk);
      }
    }
    lk.unlock();
    iters = job.iters;
    if (job.rc) return fail(job.rc, job.msg);
    return RVE_OK;
  }

  // CG iterations of up to kMaxBatch same-description handles (fused z passes, strain
  // control) as launches over all of them: block z of each kernel works on handle z, whose
  // buffers lie slotd[z] bytes from the first handle's; the first handle's stream carries
  // the launches, after every handle's set-up and before its next work.
  static void run_batch(std::vector<CgJob*>& jobs) {
    const int B = (int)jobs.size();
    rve_s* h0 = jobs[0]->h;
    Ops<R> o(h0);
    hipStream_t st = h0->st;
    auto fail_all = [&](int rc, const std::string& m) {
      for (CgJob* j : jobs) { j->rc = rc; j->msg = m; }
    };
    if (!h0->cg_done &&
        hipEventCreateWithFlags(&h0->cg_done, hipEventDisableTiming) != hipSuccess) {
      fail_all(RVE_E_DEVICE, "event creation failed");
      return;
    }
    long long d[kMaxBatch];
    for (int j = 0; j < B; ++j) {
      d[j] = (long long)(jobs[j]->h->base - h0->base);
      if (j && hipStreamWaitEvent(st, jobs[j]->h->cg_ready, 0) != hipSuccess) {
        fail_all(RVE_E_DEVICE, "stream wait failed");
        return;
      }
    }
    // (pageable source: staged before the call returns)
    if (hipMemcpyAsync(h0->slotd, d, (size_t)B * 8, hipMemcpyHostToDevice, st) != hipSuccess) {
      fail_all(RVE_E_DEVICE, "slot table upload failed");
      return;
    }
    Plans pb = h0->pl;
    pb.g.sd = h0->slotd;
    pb.nslot = B;
    C *x = o.v(0), *z = o.v(2), *p = o.v(3), *q = o.v(4), *b = o.v(5);
    double* sc = h0->scal;
    const double* stop = sc + SC_FLAG;
    double* cg_part = h0->partial + cg_partial_offset(h0->g);
    int nb_cg = 0;
    auto check_of = [&](int k) {
      return CgCheck{cg_part, nb_cg, SC_FLAG, SC_TOL2, SC_RRN, SC_RZ0 + ((k + 1) & 1)};
    };
    auto enqueue_iter = [&](int k) {
      const int cur = SC_RZ0 + (k & 1), prv = SC_RZ0 + ((k + 1) & 1);
      const int ia = (k == 0) ? SC_ZERO : cur, ib = (k == 0) ? SC_ONE : prv;
      C* pold = (k & 1) ? b : p;
      C* pk = (k & 1) ? p : b;
      if (k == 0) {
        launch_zgrad_inv<R>(pb, z, pold, pk, o.NH, sc, ia, ib, o.W, st, stop);
      } else if (cg_check_inline_mode()) {
        launch_zgrad_inv<R>(pb, z, pold, pk, o.NH, sc, ia, ib, o.W, st, stop, check_of(k - 1));
      } else {
        launch_cg_check_tail(sc, check_of(k - 1), st, h0->slotd, B);
        launch_zgrad_inv<R>(pb, z, pold, pk, o.NH, sc, ia, ib, o.W, st, stop);
      }
      launch_fft_yz<R>(pb, o.W, o.NH, 6, 1, true, st, stop);
      launch_x_tangent<R>(pb, o.W, o.NH, o.gK(), 1.0 / (double)o.N, st, stop);
      launch_fft_yz<R>(pb, o.W, o.NH, 6, 1, false, st, stop);
      const int nbd = launch_zdiv_fwd<R>(pb, o.W, q, pk, o.NH, h0->partial, st, stop);
      nb_cg = launch_cg_step<R>(pb, x, pk, q, z, o.NH, sc + SC_KBAR, sc, cur, SC_PQ, cg_part, st,
                                stop, h0->partial, nbd, SC_FLAG, SC_ITER, kCgMaxBlocks, nullptr);
    };
    const int maxk = h0->d.max_krylov;
    std::vector<double> rr_ref(B), it_ref(B, 0.0);
    for (int j = 0; j < B; ++j) rr_ref[j] = jobs[j]->h->hs[SC_BB];
    int queued = 0, batch = 4;
    bool all_done = false;
    while (queued < maxk) {
      const int nq = std::min(batch, maxk - queued);
      for (int kk = 0; kk < nq; ++kk) enqueue_iter(queued + kk);
      queued += nq;
      launch_cg_check_tail(sc, check_of(queued - 1), st, h0->slotd, B);
      for (int j = 0; j < B; ++j) {
        rve_s* hj = jobs[j]->h;
        if (hipMemcpyAsync(hj->hs + SC_RZ0, hj->scal + SC_RZ0,
                           (SC_RRN - SC_RZ0 + 1) * sizeof(double), hipMemcpyDeviceToHost,
                           st) != hipSuccess) {
          fail_all(RVE_E_DEVICE, "scalar read failed");
          return;
        }
      }
      if (hipStreamSynchronize(st) != hipSuccess || hipGetLastError() != hipSuccess) {
        fail_all(RVE_E_DEVICE, "HIP error in the batched CG iterations");
        return;
      }
      // next batch: the iterations the slowest unconverged solve still needs (as in pcg)
      all_done = true;
      int next = 4;
      batch = std::min(2 * batch, 16);
      for (int j = 0; j < B; ++j) {
        const double* hs = jobs[j]->h->hs;
        if (hs[SC_FLAG] != 0.0) continue;
        all_done = false;
        const double rr = hs[SC_RRN], its = hs[SC_ITER];
        int want = batch;
        if (its > it_ref[j] && rr > 0.0 && rr < rr_ref[j]) {
          const double rate = std::log(rr / rr_ref[j]) / (its - it_ref[j]);
          const double need = std::log(hs[SC_TOL2] / rr) / rate;
          if (std::isfinite(need)) want = std::max(4, std::min(16, (int)std::ceil(need) + 2));
        }
        next = std::max(next, want);
        rr_ref[j] = rr;
        it_ref[j] = its;
      }
      batch = next;
      if (all_done) break;
    }
    for (CgJob* j : jobs) {
      const double* hs = j->h->hs;
      j->h->batch_peak = std::max(j->h->batch_peak, B);
      j->iters = (int)hs[SC_ITER];
      if (hs[SC_FLAG] == 1.0) j->rc = RVE_OK;
      else if (hs[SC_FLAG] == 2.0) { j->rc = RVE_E_NOCONV; j->msg = "momentum CG breakdown"; }
      else { j->rc = RVE_E_NOCONV; j->msg = "momentum Krylov solver reached max_krylov"; }
    }
    // the other handles' streams resume after the batch
    if (hipEventRecord(h0->cg_done, st) != hipSuccess) {
      fail_all(RVE_E_DEVICE, "event record failed");
      return;
    }
    for (int j = 1; j < B; ++j)
      if (hipStreamWaitEvent(jobs[j]->h->st, h0->cg_done, 0) != hipSuccess)
        fail_all(RVE_E_DEVICE, "stream wait failed");
  }

  // mean tangent from the constitutive sums
  void kbar() { launch_rscale(21, h->scal + SC_K, 1.0 / (double)N, h->scal + SC_KBAR, st); }

  int constitutive(const double* deps, double t, const double* phi) {
    Material m = mat(0.0);
    m.dt = cur_dt;
    const int nb = launch_constitutive<R>(N, h->eps, deps, t, h->epsp, h->gslip, h->grain,
                                          h->gtab, h->sig, phi, gK(), h->gw, h->cf, m,
                                          h->partial, h->failc, st, h->ps_sig, h->ps_rec);
    launch_reduce(h->partial, nb, RED_CONST, 0, h->scal + SC_K, st);
    return RVE_OK;
  }
  double cur_dt = 0.0;
  Material mat(double dt) const {
    Material m;
    m.dt = dt; m.gdot0 = h->d.gdot0; m.nexp = h->d.n_exp; m.kres = h->d.k_res;
    m.h_lin = h->d.h_lin; m.lambda_ssd = h->d.lambda_ssd; m.xi_store = h->d.xi_store;
    m.G_crit = h->d.G_crit; m.ell = h->d.ell; m.Gc = h->d.Gc; m.burgers = h->d.burgers;
    const double ne = h->d.n_exp;
    m.nexp_int = (ne == std::floor(ne) && ne >= 1.0 && ne <= 64.0) ? (int)ne : 0;
    m.flow = h->d.material == RVE_MAT_DUNNE ? FLOW_DUNNE : FLOW_POWER;
    const double kT = h->d.k_B * h->d.T;
    m.A = m.flow == FLOW_DUNNE
              ? h->d.rho_m * h->d.burgers * h->d.burgers * h->d.v_D * std::exp(-h->d.dF / kT)
              : 0.0;
    m.beta = m.flow == FLOW_DUNNE ? h->d.dV / kT : 0.0;
    m.mu_b = h->d.mu * h->d.burgers;
    return m;
  }

  // Preconditioned CG on B du = c (c in cg[5]); solution in cg[0].  Iterations are
  // enqueued in batches; the convergence test runs on the device and turns the rest of
  // a batch into no-ops, so the host synchronises once per batch.
  int pcg(int& iters) {
    C *x = v(0), *z = v(2), *p = v(3), *q = v(4), *b = v(5);
    const size_t bytes = (size_t)3 * NH * sizeof(C);
    double* sc = h->scal;
    launch_zero(x, bytes, st);
    launch_zero(p, bytes, st);      // the first iteration forms p = z + 0 * p
    int nb = launch_sdot<R>(h->pl, b, b, NH, 3, h->partial, st);
    launch_reduce(h->partial, nb, 1, 0, sc + SC_BB, st);
    // z = M r with r = b; the steps update z in place (r is not stored)
    nb = launch_precond<R>(h->pl, b, z, NH, sc + SC_KBAR, h->partial, st, nullptr, m0());
    launch_reduce(h->partial, nb, 1, 0, sc + SC_RZ0, st);
    int rc = sync_read(h, SC_BB, 1);
    if (rc) return rc;
    const double bb = h->hs[SC_BB];
    iters = 0;
    if (!(bb > 0.0)) return std::isfinite(bb) ? RVE_OK : fail(RVE_E_NOCONV, "non-finite residual");
    h->hs[SC_FLAG] = 0.0;
    h->hs[SC_ITER] = 0.0;
    h->hs[SC_TOL2] = h->d.tol_lin * h->d.tol_lin * bb;
    h->hs[SC_ZERO] = 0.0;
    h->hs[SC_ONE] = 1.0;
    HIPCHK(hipMemcpyAsync(sc + SC_FLAG, h->hs + SC_FLAG, 3 * sizeof(double), hipMemcpyHostToDevice, st));
    HIPCHK(hipMemcpyAsync(sc + SC_ZERO, h->hs + SC_ZERO, 2 * sizeof(double), hipMemcpyHostToDevice, st));
    const double* stop = sc + SC_FLAG;
    // With the fused z passes the direction alternates between two buffers (the
    // right-hand side is no longer needed once z = M b is formed): each iteration reads p_old and
    // writes p_new while other blocks still read p_old.
    const bool fz = fused_z_available<R>(h->pl);
    // inside a pool tick, the same-size handles' solves advance in shared launches
    if (h->cg_group && mask == 0 && fz && h->time_xt == 0) return pcg_batched(iters);
    // the captured graphs hold the macro launches of one stress-control mask
    if (h->graph_mask != mask) {
      for (auto& ex : h->cg_exec)
        if (ex) { (void)hipGraphExecDestroy(ex); ex = nullptr; }
      h->graph_mask = mask;
    }
    const long long zst = (long long)h->g.n1h * h->g.n2;   // z stride of the half spectrum
    // With the fused z passes an iteration is six launches: the convergence test of the
    // previous iteration runs inside the inverse z pass and the sum of <p, q> inside the
    // CG step (each block reduces the previous kernel's partials itself).
    double* cg_part = h->partial + cg_partial_offset(h->g);
    int nb_cg = 0;
    auto check_of = [&](int k) {        // the test of iteration k (after its CG step)
      return CgCheck{cg_part, nb_cg, SC_FLAG, SC_TOL2, SC_RRN, SC_RZ0 + ((k + 1) & 1)};
    };
    // the launches of CG iteration k (those of k >= 1 depend on the parity of k only)
    auto enqueue_iter = [&](int k) {
      const int cur = SC_RZ0 + (k & 1), prv = SC_RZ0 + ((k + 1) & 1);
      // p = z + beta p (beta = rz_k / rz_{k-1}, 0 on the first iteration), gradient
      const int ia = (k == 0) ? SC_ZERO : cur, ib = (k == 0) ? SC_ONE : prv;
      if (fz) {
        C* pold = (k & 1) ? b : p;
        C* pk = (k & 1) ? p : b;
        if (k == 0) {
          launch_zgrad_inv<R>(h->pl, z, pold, pk, NH, sc, ia, ib, W, st, stop);
        } else if (cg_check_inline_mode()) {
          launch_zgrad_inv<R>(h->pl, z, pold, pk, NH, sc, ia, ib, W, st, stop, check_of(k - 1));
        } else {      // the test writes <r, z> into sc[ia] and the flag the pass stops on
          launch_cg_check_tail(sc, check_of(k - 1), st);
          launch_zgrad_inv<R>(h->pl, z, pold, pk, NH, sc, ia, ib, W, st, stop);
        }
        if (mask)   // macro strain along the (0, 0) z column (z already inverse transformed)
          launch_macro_strain<R>(W, NH, pk, NH, s_mac, 0.0, mask, h->g.n3, zst, nullptr, st, stop);
        launch_fft_yz<R>(h->pl, W, NH, 6, 1, true, st, stop);
        timed_x_tangent(k, stop);
        launch_fft_yz<R>(h->pl, W, NH, 6, 1, false, st, stop);
        // q = -i xi~ . sigma^ with the partials of <p, q>; the step sums them
        int nbd = launch_zdiv_fwd<R>(h->pl, W, q, pk, NH, h->partial, st, stop);
        if (mask) {  // q(0) from the macro stress (z still spatial), its term of <p, q>
          launch_macro_stress<R>(W, NH, q, pk, NH, s_mac, mask, h->g.n3, zst, h->partial + nbd, st,
                                 stop);
          ++nbd;
        }
        nb_cg = launch_cg_step<R>(h->pl, x, pk, q, z, NH, sc + SC_KBAR, sc, cur, SC_PQ,
                                  cg_part, st, stop, h->partial, nbd, SC_FLAG, SC_ITER,
                                  kCgMaxBlocks, m0());
        return;
      }
      // unfused operator (grids without a register DFT length)
      launch_grad_cgp<R>(h->pl, p, z, NH, sc, ia, ib, W, st, stop);
      if (mask) launch_macro_strain<R>(W, NH, p, NH, s_mac, 0.0, mask, 1, 0, nullptr, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 6, 2, true, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 6, 1, true, st, stop);
      timed_x_tangent(k, stop);
      launch_fft_yz<R>(h->pl, W, NH, 6, 1, false, st, stop);
      launch_fft_yz<R>(h->pl, W, NH, 6, 2, false, st, stop);
      // q = -i xi~ . sigma^ and <p, q> into sc[SC_PQ] (flag 2 if not positive)
      nb = launch_div_dot<R>(h->pl, W, q, p, NH, h->partial, st, stop);
      if (mask) {
        launch_macro_stress<R>(W, NH, q, p, NH, s_mac, mask, 1, 0, h->partial + nb, st, stop);
        ++nb;
      }
      launch_reduce_pq(h->partial, nb, sc, SC_PQ, SC_FLAG, st);
      // x and z updates, <r, r>, <r, z> and the convergence test
      nb = launch_cg_step<R>(h->pl, x, p, q, z, NH, sc + SC_KBAR, sc, cur, SC_PQ,
                             h->partial, st, stop, nullptr, 0, 0, 0, 1 << 30, m0());
      launch_reduce_check(h->partial, nb, sc, SC_ITER, prv, SC_RRN, SC_FLAG, SC_TOL2, st);
    };
    int queued = 0, batch = 4, it_ref = 0;
    double rr_ref = bb;
    while (queued < h->d.max_krylov) {
      const int nq = std::min(batch, h->d.max_krylov - queued);
      for (int kk = 0; kk < nq; ++kk) {
        const int k = queued + kk;
        // timed iterations run eagerly (their launch records an event pair)
        if (k == 0 || !h->use_graphs || timed_iter(k)) {
          enqueue_iter(k);
          continue;
        }
        // iterations k >= 1 replay the captured graph of their parity
        hipGraphExec_t& ex = h->cg_exec[k & 1];
        if (!ex) {
          hipGraph_t gr = nullptr;
          bool ok = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) == hipSuccess;
          if (ok) {
            enqueue_iter(k);
            ok = hipStreamEndCapture(st, &gr) == hipSuccess && gr != nullptr;
          }
          if (ok) ok = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0) == hipSuccess;
          if (gr) (void)hipGraphDestroy(gr);
          if (!ok) {                         // no graphs on this stream: launch eagerly
            (void)hipGetLastError();
            ex = nullptr;
            h->use_graphs = false;
            enqueue_iter(k);
            continue;
          }
        }
        HIPCHK(hipGraphLaunch(ex, st));
      }
      queued += nq;
      if (fz) launch_cg_check_tail(sc, check_of(queued - 1), st);
      rc = sync_read(h, SC_RZ0, SC_RRN - SC_RZ0 + 1);
      if (rc) return rc;
      iters = (int)h->hs[SC_ITER];
      if ((rc = harvest_x_tangent(iters))) return rc;
      if (g_debug)
        std::fprintf(stderr, "  pcg queued %d ran %d flag %g rr %.3e tol2 %.3e pq %.3e\n", queued, iters,
                     h->hs[SC_FLAG], h->hs[SC_RRN], h->hs[SC_TOL2], h->hs[SC_PQ]);
      if (g_debug) std::fprintf(stderr, "    rz0 %.6e rz1 %.6e\n", h->hs[SC_RZ0], h->hs[SC_RZ1]);
      if (h->hs[SC_FLAG] == 1.0) return RVE_OK;
      if (h->hs[SC_FLAG] == 2.0) return fail(RVE_E_NOCONV, "momentum CG breakdown");
      // next batch: the iterations the residual's recent rate of decrease still needs,
      // plus two, at least 4 and at most 32 (the launches of a batch that follow
      // convergence return at once; each batch costs one host round trip; 32 measured
      // 0.1-0.4 % faster than 16 at 128^3)
      const double rr = h->hs[SC_RRN];
      batch = std::min(2 * batch, 32);
      if (iters > it_ref && rr > 0.0 && rr < rr_ref) {
        const double rate = std::log(rr / rr_ref) / (double)(iters - it_ref);   // < 0
        const double need = std::log(h->hs[SC_TOL2] / rr) / rate;
        if (std::isfinite(need)) batch = std::max(4, std::min(32, (int)std::ceil(need) + 2));
      }
      rr_ref = rr;
      it_ref = iters;
    }
    return fail(RVE_E_NOCONV, "momentum Krylov solver reached max_krylov");
  }
};

// Phase-field balance with the pre-set crack held at phi = 1 (Dirichlet option): phi =
// X + 1_crack, X from CG on P A P u = P (2S - A 1_crack), A = (1 + 2S) - l^2 lap, with the
// restricted preconditioner P (1 - l^2 lap)^-1 P; P restricts to the voxels that can slip.
// The Laplacian and the preconditioner are FFT round trips; convergence control on the
// device in batches, as in the other Krylov loops.  Writes phi before the clamp into X
// (rbuf[0, N)); adds the matrix-vector products to *iters.
template <typename R>
int pf_dirichlet_solve(rve_s* h, Ops<R>& o, int* iters) {
  typedef cplx<R> C;
  hipStream_t st = h->st;
  const long long N = h->g.nvox;
  const double invN = 1.0 / (double)N;
  C* W1 = (C*)h->spec;
  double* X = h->rbuf;
  double *Rr = h->rbuf + N, *Z = h->rbuf + 2 * N, *P = h->rbuf + 3 * N, *Wv = h->rbuf + 4 * N;
  double *Q = h->rbuf + 5 * N, *Y = h->rbuf + 6 * N;
  double* sc = h->scal;
  // out = F^-1 f(xi) F in, f = l^2 |xi|^2 (lap) or (1 + l^2 |xi|^2)^-1
  auto spec_op = [&](const double* in, double* outp, int lap, const double* stp) {
    launch_x_r2c<R>(h->pl, in, true, N, nullptr, 0.0, W1, o.NH, 1, st, stp);
    launch_fft_yz<R>(h->pl, W1, o.NH, 1, 1, false, st, stp);
    launch_fft_yz<R>(h->pl, W1, o.NH, 1, 2, false, st, stp);
    launch_pf_scale<R>(h->pl, W1, h->d.ell, invN, st, stp, lap);
    launch_fft_yz<R>(h->pl, W1, o.NH, 1, 2, true, st, stp);
    launch_fft_yz<R>(h->pl, W1, o.NH, 1, 1, true, st, stp);
    launch_x_c2r<R>(h->pl, W1, o.NH, outp, true, N, 1, 1.0, 0, st, stp);
  };
  int rc;
  launch_zero(X, N * 8, st);
  launch_pfd(N, 1, nullptr, nullptr, nullptr, h->gslip, Y, st);
  spec_op(Y, Wv, 1, nullptr);
  launch_pfd(N, 3, Y, Wv, h->S, h->gslip, Rr, st);
  int nb = launch_rdot(N, Rr, Rr, h->partial, st);
  launch_reduce(h->partial, nb, 1, 0, sc + SC_BB, st);
  if ((rc = sync_read(h, SC_BB, 1))) return rc;
  const double bb = h->hs[SC_BB];
  if (!std::isfinite(bb)) return fail(RVE_E_NOCONV, "non-finite phase-field residual");
  if (bb > 0.0) {
    h->hs[SC_FLAG] = 0.0;
    h->hs[SC_ITER] = 0.0;
    h->hs[SC_TOL2] = h->d.tol_lin * h->d.tol_lin * bb;
    HIPCHK(hipMemcpyAsync(sc + SC_FLAG, h->hs + SC_FLAG, 3 * sizeof(double),
                          hipMemcpyHostToDevice, st));
    const double* stop = sc + SC_FLAG;
    spec_op(Rr, Wv, 0, nullptr);
    launch_pfd(N, 0, Wv, nullptr, nullptr, h->gslip, Z, st);
    nb = launch_rdot(N, Rr, Z, h->partial, st);
    launch_reduce(h->partial, nb, 1, 0, sc + SC_RZ0, st);
    HIPCHK(hipMemcpyAsync(P, Z, N * 8, hipMemcpyDeviceToDevice, st));
    bool ok = false;
    int queued = 0, batch = 4;
    while (queued < h->d.max_krylov) {
      const int nq = std::min(batch, h->d.max_krylov - queued);
      for (int kk = 0; kk < nq; ++kk) {
        const int k = queued + kk;
        const int cur = SC_RZ0 + (k & 1), nxt = SC_RZ0 + ((k + 1) & 1);
        spec_op(P, Wv, 1, stop);
        launch_pfd(N, 2, P, Wv, h->S, h->gslip, Q, st, stop);
        nb = launch_rdot(N, P, Q, h->partial, st, stop);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_PQ, st, stop);
        launch_pfd_axpy(N, sc, cur, SC_PQ, 1.0, P, X, st, stop);
        launch_pfd_axpy(N, sc, cur, SC_PQ, -1.0, Q, Rr, st, stop);
        nb = launch_rdot(N, Rr, Rr, h->partial, st, stop);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_RR, st, stop);
        launch_pf_check(sc, SC_FLAG, SC_ITER, SC_PQ, SC_RR, SC_TOL2, st);
        spec_op(Rr, Wv, 0, stop);
        launch_pfd(N, 0, Wv, nullptr, nullptr, h->gslip, Z, st, stop);
        nb = launch_rdot(N, Rr, Z, h->partial, st, stop);
        launch_reduce(h->partial, nb, 1, 0, sc + nxt, st, stop);
        launch_pfd_xpby(N, Z, sc, nxt, cur, P, st, stop);
      }
      queued += nq;
      if ((rc = sync_read(h, SC_FLAG, 2))) return rc;
      if (h->hs[SC_FLAG] != 0.0) {
        ok = h->hs[SC_FLAG] == 1.0;
        break;
      }
      batch = std::min(2 * batch, 16);
    }
    *iters += (int)h->hs[SC_ITER];
    if (!ok) return fail(RVE_E_NOCONV, "phase-field Krylov solver did not converge");
  }
  launch_pfd_axpy(N, nullptr, 0, 0, 1.0, Y, X, st);
  return RVE_OK;
}

// Phase-field balance (eqs. strpf, phase) at the driving state h->S (sum S, sum S^2 over
// the voxels given): PCG with the preconditioner of eq. precph, (1 + l^2 |xi|^2)^-1, one
// FFT round trip per iteration (or the Dirichlet option's solve); writes phi before the
// clamp into X = rbuf[0, N) and adds the iterations to *pf_iters.
template <typename R>
int pf_solve(rve_s* h, Ops<R>& o, double sumS, double sumS2, int* pf_iters) {
  hipStream_t st = h->st;
  const long long N = h->g.nvox;
  const double invN = 1.0 / (double)N;
  int rc = RVE_OK;
  double* X = h->rbuf;
  double *Rr = h->rbuf + N, *Z = h->rbuf + 2 * N, *P = h->rbuf + 3 * N, *Wv = h->rbuf + 4 * N;
  launch_zero(X, N * 8, st);
  if (h->d.pf_dirichlet && h->n_preset > 0) {
    if ((rc = pf_dirichlet_solve<R>(h, o, pf_iters))) return rc;
  } else if (sumS > 0.0) {
    typedef cplx<R> C;
    C* W1 = (C*)h->spec;
    const double bb = 4.0 * sumS2;
    const double tol2 = h->d.tol_lin * h->d.tol_lin * bb;
    launch_rscale(N, h->S, 2.0, Rr, st);
    // convergence control on the device, as in the momentum CG: iterations are enqueued
    // in batches and the test turns the rest of a batch into no-ops
    double* sc = h->scal;
    h->hs[SC_FLAG] = 0.0;
    h->hs[SC_ITER] = 0.0;
    h->hs[SC_TOL2] = tol2;
    HIPCHK(hipMemcpyAsync(sc + SC_FLAG, h->hs + SC_FLAG, 3 * sizeof(double),
                          hipMemcpyHostToDevice, st));
    const double* stop = sc + SC_FLAG;
    auto prec = [&](const double* in, double* outp, const double* stp) {
      launch_x_r2c<R>(h->pl, in, true, N, nullptr, 0.0, W1, o.NH, 1, st, stp);
      launch_fft_yz<R>(h->pl, W1, o.NH, 1, 1, false, st, stp);
      launch_fft_yz<R>(h->pl, W1, o.NH, 1, 2, false, st, stp);
      launch_pf_scale<R>(h->pl, W1, h->d.ell, invN, st, stp);
      launch_fft_yz<R>(h->pl, W1, o.NH, 1, 2, true, st, stp);
      launch_fft_yz<R>(h->pl, W1, o.NH, 1, 1, true, st, stp);
      launch_x_c2r<R>(h->pl, W1, o.NH, outp, true, N, 1, 1.0, 0, st, stp);
    };
    prec(Rr, Z, nullptr);
    int nb = launch_rdot(N, Rr, Z, h->partial, st);
    launch_reduce(h->partial, nb, 1, 0, sc + SC_RZ0, st);
    HIPCHK(hipMemcpyAsync(P, Z, N * 8, hipMemcpyDeviceToDevice, st));
    HIPCHK(hipMemcpyAsync(Wv, Rr, N * 8, hipMemcpyDeviceToDevice, st));
    bool ok = false;
    int queued = 0, batch = 4;
    while (queued < h->d.max_krylov) {
      const int nq = std::min(batch, h->d.max_krylov - queued);
      for (int kk = 0; kk < nq; ++kk) {
        const int k = queued + kk;
        const int cur = SC_RZ0 + (k & 1), nxt = SC_RZ0 + ((k + 1) & 1);
        nb = launch_pf_pq(N, P, Wv, h->S, h->partial, st, stop);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_PQ, st, stop);
        nb = launch_pf_xr(N, X, Rr, P, Wv, h->S, sc, cur, SC_PQ, h->partial, st, stop);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_RR, st, stop);
        launch_pf_check(sc, SC_FLAG, SC_ITER, SC_PQ, SC_RR, SC_TOL2, st);
        prec(Rr, Z, stop);
        nb = launch_rdot(N, Rr, Z, h->partial, st, stop);
        launch_reduce(h->partial, nb, 1, 0, sc + nxt, st, stop);
        launch_pf_pw(N, P, Wv, Z, Rr, sc, nxt, cur, st, stop);
      }
      queued += nq;
      if ((rc = sync_read(h, SC_FLAG, 2))) return rc;
      if (h->hs[SC_FLAG] != 0.0) {
        ok = h->hs[SC_FLAG] == 1.0;
        break;
      }
      batch = std::min(2 * batch, 16);
    }
    *pf_iters += (int)h->hs[SC_ITER];
    if (!ok) return fail(RVE_E_NOCONV, "phase-field Krylov solver did not converge");
  }
  return RVE_OK;
}

template <typename R>
int run_increment(rve_s* h, const double de_in[6], const double* dsig, int mask, double dt,
                  rve_stats* out) {
  Ops<R> o(h);
  o.cur_dt = dt;
  hipStream_t st = h->st;
  const long long N = h->g.nvox;
  const double invN = 1.0 / (double)N;
  // mixed control: the stress-controlled components of the macro strain are unknowns;
  // their target macro stress is that of t plus the increment (Mandel values)
  static constexpr double kRt2 = 1.41421356237309504880;
  double de[6], tgt[6], Ecur[6];
  for (int c = 0; c < 6; ++c) {
    const bool f = (mask >> c) & 1;
    const double w = c < 3 ? 1.0 : kRt2;
    de[c] = f ? 0.0 : de_in[c];
    tgt[c] = f ? w * (h->msig_t[c] + dsig[c]) : 0.0;
    Ecur[c] = f ? w * h->meps_t[c] : 0.0;      // stress-controlled macro strain (Mandel)
  }
  o.mask = mask;
  {
    const double lmax = h->d.h * (double)std::max(h->g.n1, std::max(h->g.n2, h->g.n3));
    o.s_mac = (double)N * 6.283185307179586476925286766559 / lmax;
  }
  // external work of the prescribed macro stress per voxel, - sigma*_F . E_F
  auto ext = [&](const double* E, double t, const double* dE) {
    double a = 0.0;
    for (int c = 0; c < 6; ++c) a -= tgt[c] * (E[c] + (dE ? t * dE[c] : 0.0));
    return a;
  };
  rve_stats s;
  std::memset(&s, 0, sizeof(s));
  const double t0 = now_ms();
  int rc;
  h->batch_peak = 1;
  const bool coupled = h->d.gnd_coupling != 0;
  // transactional copies of the state at time t
  if (coupled) HIPCHK(hipMemcpyAsync(h->g_n, h->gslip, N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->eps_t, h->eps, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->sig_t, h->sig, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->phi_t, h->phi, N * 8, hipMemcpyDeviceToDevice, st));
  launch_zero(h->failc, sizeof(int), st);
  // eps_0 = eps_t + d eps_bar (uniform)
  launch_add_uniform(N, h->eps, de, st);
  HIPCHK(hipMemcpyAsync(h->eps_prev, h->eps, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->phi_prev, h->phi_t, N * 8, hipMemcpyDeviceToDevice, st));

  bool converged = false;
  double omega = 0.5;        // relaxation of the coupled strength (Aitken; first pass 1/2)
  for (int it = 0; it < h->d.max_stag && !converged; ++it) {
    s.stag_iters = it + 1;
    // ---- momentum balance at phi_prev (Newton + PCG, line search on the energy) ----
    double tc = now_ms();
    o.constitutive(nullptr, 0.0, h->phi_prev);
    if ((rc = sync_read(h, SC_K, 28))) return rc;
    s.ms_constitutive += now_ms() - tc;
    double Pi = h->hs[SC_K + 21] * invN + ext(Ecur, 0.0, nullptr);
    bool newton_ok = false;
    for (int nit = 0; nit < h->d.max_newton; ++nit) {
      s.newton_iters++;
      double tk = now_ms();
      o.kbar();
      if (mask) launch_macro_prec(h->scal + SC_KBAR, o.s_mac * o.s_mac, mask, h->scal + SC_M0, st);
      // c = i xi~ . F{ g sigma } (plane stress: the condensed stress)
      o.fwd(h->ps_sig ? h->ps_sig : h->sig, true, N, 6, o.W, h->phi_prev);
      launch_div<R>(h->pl, o.W, o.NH, o.v(5), o.NH, 1.0, st);
      launch_herm_proj<R>(h->pl, o.v(5), o.NH, 3, st);
      // zero bin: -s (sum g sigma - N sigma*) on the stress-controlled components
      if (mask) launch_macro_rhs<R>(o.W, o.NH, o.v(5), o.NH, o.s_mac, (double)N, tgt, mask, st);
      int kit = 0;
      rc = h->d.krylov == RVE_KRYLOV_GMRES ? o.gmres(kit) : o.pcg(kit);
      s.krylov_iters += kit;
      if (rc) { s.ms_mech_krylov += now_ms() - tk; goto fail_out; }
      // deps = F^-1{ sym(i xi~ (x) du) }
      launch_sym_grad<R>(h->pl, o.v(0), o.NH, o.W, o.NH, st);
      if (mask)   // + the macro strain increment at the zero bin, recorded in SC_DE
        launch_macro_strain<R>(o.W, o.NH, o.v(0), o.NH, o.s_mac, o.s_mac * invN, mask, 1, 0,
                               h->scal + SC_DE, st);
      o.inv(o.W, 6, h->deps, true, N, invN, 0);
      if (h->ps_rec) launch_plane_recover(N, h->deps, h->ps_rec, st);
      launch_slope(N, h->sig, h->deps, h->phi_prev, h->d.k_res, h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), 1, 0, h->scal + SC_MISC, st);
      s.ms_mech_krylov += now_ms() - tk;
      // backtracking on the incremental energy; its first trial (t = 1) is evaluated
      // whatever the slope, so it is enqueued before the host reads the slope, and one
      // round trip returns the slope, the trial's sums (and the macro strain increment)
      tc = now_ms();
      o.constitutive(h->deps, 1.0, h->phi_prev);
      static_assert(SC_K == 0 && SC_MISC > SC_K + 28 && SC_DE > SC_MISC, "scalar slot order");
      if ((rc = sync_read(h, SC_K, (mask ? SC_DE + 6 : SC_MISC + 1) - SC_K))) return rc;
      double slope = h->hs[SC_MISC] * invN;
      double dE[6] = {0, 0, 0, 0, 0, 0};
      if (mask) {
        for (int c = 0; c < 6; ++c) dE[c] = h->hs[SC_DE + c];
        slope += ext(dE, 0.0, nullptr);          // - sigma*_F . dE_F
      }
      double t = 1.0, Pit = 0.0;
      bool acc = false;
      for (int ls = 0; ls < 40; ++ls) {
        if (ls > 0) {
          o.constitutive(h->deps, t, h->phi_prev);
          if ((rc = sync_read(h, SC_K, 28))) return rc;
        }
        Pit = h->hs[SC_K + 21] * invN + ext(Ecur, t, dE);
        if (Pit - Pi <= 1e-4 * t * slope + 1e-13 * std::fabs(Pi)) { acc = true; break; }
        t *= 0.5;
        s.ls_cuts++;
      }
      s.ms_constitutive += now_ms() - tc;
      if (!acc) { rc = fail(RVE_E_NOCONV, "Newton line search failed"); goto fail_out; }
      Pi = Pit;
      for (int c = 0; c < 6; ++c) Ecur[c] += t * dE[c];
      launch_eps_update(N, h->eps, h->deps, t, h->eps_t, h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), 2, 1, h->scal + SC_MISC, st);
      if ((rc = sync_read(h, SC_MISC, 2))) return rc;
      const double num = h->hs[SC_MISC], den = h->hs[SC_MISC + 1];
      if (num <= h->d.tol_newton * den || num == 0.0) { newton_ok = true; break; }
    }
    if (!newton_ok) { rc = fail(RVE_E_NOCONV, "Newton reached max_newton"); goto fail_out; }
    // ---- phase field at eps_i ----
    {
      double tp = now_ms();
      Material m = o.mat(dt);
      launch_source(N, h->eps, h->sig, h->epsp, h->gslip, h->grain, h->gtab, h->wp, h->trig,
                    h->wcrit, h->S, h->wep, m, h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), RED_SOURCE, 0, h->scal + SC_MISC, st);
      if ((rc = sync_read(h, SC_MISC, 2))) return rc;
      const double sumS = h->hs[SC_MISC], sumS2 = h->hs[SC_MISC + 1];
      if ((rc = pf_solve<R>(h, o, sumS, sumS2, &s.pf_iters))) {
        s.ms_phase_field += now_ms() - tp;
        if (rc == RVE_E_NOCONV) goto fail_out;
        return rc;
      }
      double* X = h->rbuf;
      launch_clamp(N, X, h->phi_t, h->phi, st);
      launch_stag_norms(N, h->eps, h->eps_prev, h->eps_t, h->phi, h->phi_prev, h->phi_t,
                        h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), 4, 1, h->scal + SC_MISC, st);
      if ((rc = sync_read(h, SC_MISC, 4))) return rc;
      auto ratio = [](double a, double b) { return a == 0.0 ? 0.0 : (b > 0.0 ? a / b : INFINITY); };
      const double re = ratio(h->hs[SC_MISC], h->hs[SC_MISC + 1]);
      const double rp = ratio(h->hs[SC_MISC + 2], h->hs[SC_MISC + 3]);
      HIPCHK(hipMemcpyAsync(h->eps_prev, h->eps, 6 * N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(h->phi_prev, h->phi, N * 8, hipMemcpyDeviceToDevice, st));
      s.ms_phase_field += now_ms() - tp;
      double rg = 0.0;
      if (coupled) {
        // the end-of-increment densities of this pass's slip (the Nye tensor of the trial
        // plastic distortion, non-local) and the Taylor strength of the next pass
        Material mc = o.mat(dt);
        launch_trial_hardening(N, h->sig, h->gslip, h->beta, h->rho_ssd, h->grain, h->gtab, mc,
                               h->rbuf, h->rho_ssd_tr, st);
        typedef cplx<R> C;
        C* B9 = (C*)h->spec;
        o.fwd(h->rbuf, true, N, 9, B9);
        launch_curl_reg<R>(h->pl, B9, o.NH, h->d.ell_fp, invN, st);
        o.inv(B9, 9, h->rbuf, true, N, 1.0, 0);
        launch_gnd(N, h->rbuf, h->grain, h->gtab, h->Q81, h->d.burgers, h->rho_gnd_tr, st);
        launch_taylor_next(N, h->gslip, h->g_n, h->rho_ssd_tr, h->rho_gnd_tr, h->grain, h->gtab,
                           mc.mu_b, h->g_next, h->partial, st);
        const int nbv = voxel_grid(N);
        launch_reduce(h->partial, nbv, 2, 1, h->scal + SC_MISC, st);
        launch_aitken_dots(N, h->gslip, h->g_next, h->g_res, it == 0, h->partial + 2LL * nbv, st);
        launch_reduce(h->partial + 2LL * nbv, nbv, 2, 0, h->scal + SC_MISC + 2, st);
        if ((rc = sync_read(h, SC_MISC, 4))) return rc;
        rg = ratio(h->hs[SC_MISC], h->hs[SC_MISC + 1]);
        // Aitken's update of the relaxation factor from the last two residuals
        const double num_w = h->hs[SC_MISC + 2], den_w = h->hs[SC_MISC + 3];
        if (it > 0 && den_w > 0.0) omega = -omega * num_w / den_w;
      }
      if (g_debug)
        std::fprintf(stderr, "  stag pass %d: strain %.3e damage %.3e strength %.3e\n", it, re, rp,
                     rg);
      if (re <= h->d.tol_stag && rp <= h->d.tol_stag && rg <= h->d.tol_stag) converged = true;
      else if (coupled)   // the next pass solves the momentum balance at the relaxed strength
        launch_aitken_relax(N, h->gslip, h->g_next, h->g_res, omega, st);
    }
  }
  if (!converged) { rc = fail(RVE_E_NOCONV, "alternating minimisation reached max_stag"); goto fail_out; }
  {
    int nfail = 0;
    HIPCHK(hipMemcpyAsync(&nfail, h->failc, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    s.rm_failures = nfail;
    if (nfail > 0) { rc = fail(RVE_E_NOCONV, "return mapping did not converge"); goto fail_out; }
  }
  {
    // ---- commit ----
    double tcm = now_ms();
    Material m = o.mat(dt);
    if (coupled)      // G_s with the end-of-increment GND density
      HIPCHK(hipMemcpyAsync(h->rho_gnd, h->rho_gnd_tr, N * 8, hipMemcpyDeviceToDevice, st));
    launch_commit(N, h->sig, h->gslip, h->epsp, h->beta, h->rho_ssd, h->rho_gnd, h->wp, h->gs, h->H,
                  h->wcrit, h->trig, h->wep, h->phi, h->eps, h->grain, h->gtab, m, h->partial, st);
    const int nb = voxel_grid(N);
    launch_reduce(h->partial, nb, 13, 0, h->scal + SC_MISC, st);
    launch_reduce(h->partial + 13LL * nb, nb, 2, 1, h->scal + SC_MISC + 13, st);
    // GND density from the committed plastic distortion (used by the next increment)
    typedef cplx<R> C;
    C* B9 = (C*)h->spec;
    o.fwd(h->beta, true, N, 9, B9);
    launch_curl_reg<R>(h->pl, B9, o.NH, h->d.ell_fp, invN, st);
    o.inv(B9, 9, h->rbuf, true, N, 1.0, 0);
    launch_gnd(N, h->rbuf, h->grain, h->gtab, h->Q81, h->d.burgers, h->rho_gnd, st);
    if (m.flow == FLOW_DUNNE)
      launch_taylor(N, h->gslip, h->rho_ssd, h->rho_gnd, h->grain, h->gtab, m.mu_b, st);
    if ((rc = sync_read(h, SC_MISC, 15))) return rc;
    for (int c = 0; c < 6; ++c) {
      s.macro_stress[c] = h->hs[SC_MISC + c] * invN;
      s.macro_strain[c] = h->hs[SC_MISC + 6 + c] * invN;
    }
    s.n_triggered = h->hs[SC_MISC + 12];
    s.max_phi = h->hs[SC_MISC + 13];
    s.max_phi_slip = h->hs[SC_MISC + 14];
    for (int c = 0; c < 6; ++c) {
      h->msig_t[c] = s.macro_stress[c];
      h->meps_t[c] = s.macro_strain[c];
    }
    s.ms_commit = now_ms() - tcm;
  }
  s.ms_total = now_ms() - t0;
  s.cg_batch = h->batch_peak;
  if (out) *out = s;
  return RVE_OK;

fail_out:
  // roll back to time t
  {
    std::string msg = g_err;
    if (coupled) (void)hipMemcpyAsync(h->gslip, h->g_n, N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(h->eps, h->eps_t, 6 * N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(h->sig, h->sig_t, 6 * N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(h->phi, h->phi_t, N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
    s.ms_total = now_ms() - t0;
    if (out) *out = s;
    g_err = msg;
  }
  return rc;
}


// One finite-strain increment (Algorithm 1; Sec. 2.1 kinematics, eqs. fdef, newton,
// precf): Newton on the displacement with full steps, halved while the preconditioned
// residual |M c| grows (this integration has no incremental energy), the paper's GMRES,
// the stop test max|t grad du| <= tol_newton max|F_i - F_t|; the phase field and the
// alternating minimisation as in the small-strain increment; the commit of Fp, the
// history and the GND density of the regularised curl of Fp.
int run_increment_fs(rve_s* h, const double dF9[9], double dt, rve_stats* out) {
  typedef cplx<double> C;
  Ops<double> o(h);
  o.fs = true;
  o.cur_dt = dt;
  const long long N = h->g.nvox;
  const double invN = 1.0 / (double)N;
  hipStream_t st = h->st;
  rve_stats s;
  std::memset(&s, 0, sizeof(s));
  const double t0 = now_ms();
  int rc;
  const Material m = o.mat(dt);
  // transactional copies of the state at time t (sig: the return map's warm starts)
  HIPCHK(hipMemcpyAsync(h->fs_Ft, h->fs_F, 9 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->sig_t, h->sig, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->phi_t, h->phi, N * 8, hipMemcpyDeviceToDevice, st));
  launch_zero(h->failc, sizeof(int), st);
  launch_fs_add_uniform(N, h->fs_F, dF9, st);
  HIPCHK(hipMemcpyAsync(h->fs_Fprev, h->fs_F, 9 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->phi_prev, h->phi_t, N * 8, hipMemcpyDeviceToDevice, st));
  auto constit = [&](const double* dF, double t) {
    launch_fs_constitutive(N, h->fs_F, dF, t, h->fs_Fp, h->gslip, h->grain, h->gtab, h->sig,
                           h->phi_prev, h->fs_P, h->fs_fptr, h->fs_aux, (double*)h->gK, h->ff, m,
                           h->failc, st);
  };
  // c = i xi~_j F{ g(phi) P_ij } (eq. momentum) into cg[5], projected on real-field spectra
  auto residual = [&]() {
    o.fwd(h->fs_P, true, N, 9, o.W, h->phi_prev);
    launch_fs_div(h->pl, o.W, o.NH, o.v(5), o.NH, 1.0, st);
    launch_herm_proj<double>(h->pl, o.v(5), o.NH, 3, st);
  };
  // |M c| (Parseval), M from the mean tangent of the Newton iteration's start
  auto merit = [&](double& val) -> int {
    launch_fs_precond(h->pl, o.v(5), o.v(1), o.NH, h->scal + SC_FK, st);
    const int nb = launch_sdot<double>(h->pl, o.v(1), o.v(1), o.NH, 3, h->partial, st);
    launch_reduce(h->partial, nb, 1, 0, h->scal + SC_MISC, st);
    const int r = sync_read(h, SC_MISC, 1);
    if (r) return r;
    val = std::sqrt(h->hs[SC_MISC]);
    return RVE_OK;
  };
  bool converged = false;
  for (int it = 0; it < h->d.max_stag && !converged; ++it) {
    s.stag_iters = it + 1;
    double tc = now_ms();
    constit(nullptr, 0.0);
    residual();
    s.ms_constitutive += now_ms() - tc;
    bool newton_ok = false;
    for (int nit = 0; nit < h->d.max_newton; ++nit) {
      s.newton_iters++;
      double tk = now_ms();
      {   // mean tangent (eq. avstiff) of the current tangent field
        const int nb = launch_colsum((const double*)h->gK, N, 81, h->partial, st);
        launch_reduce(h->partial, nb, 81, 0, h->scal + SC_FK, st);
        launch_rscale(81, h->scal + SC_FK, invN, h->scal + SC_FK, st);
      }
      double m0 = 0.0;
      if ((rc = merit(m0))) return rc;
      int kit = 0;
      rc = o.gmres(kit);
      s.krylov_iters += kit;
      if (rc) { s.ms_mech_krylov += now_ms() - tk; goto fail_out; }
      // dF = F^-1{ i xi~ (x) du } (9 components)
      launch_fs_grad(h->pl, o.v(0), o.NH, o.W, o.NH, st);
      o.inv(o.W, 9, h->fs_dF, true, N, invN, 0);
      s.ms_mech_krylov += now_ms() - tk;
      tc = now_ms();
      double t = 1.0;
      bool acc = false;
      for (int ls = 0; ls < 30; ++ls) {
        constit(h->fs_dF, t);
        residual();
        double mt = 0.0;
        if ((rc = merit(mt))) return rc;
        if (mt <= m0 || m0 == 0.0) { acc = true; break; }
        t *= 0.5;
        s.ls_cuts++;
      }
      s.ms_constitutive += now_ms() - tc;
      if (!acc) {
        rc = fail(RVE_E_NOCONV, "finite-strain Newton: no step reduces the residual");
        goto fail_out;
      }
      launch_fs_update(N, h->fs_F, h->fs_dF, t, h->fs_Ft, h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), 2, 1, h->scal + SC_MISC, st);
      if ((rc = sync_read(h, SC_MISC, 2))) return rc;
      const double num = h->hs[SC_MISC], den = h->hs[SC_MISC + 1];
      if (num <= h->d.tol_newton * den || num == 0.0) { newton_ok = true; break; }
    }
    if (!newton_ok) { rc = fail(RVE_E_NOCONV, "Newton reached max_newton"); goto fail_out; }
    {   // ---- phase field at F_i ----
      double tp = now_ms();
      launch_fs_source(N, h->fs_aux, h->wp, h->trig, h->wcrit, h->S, m, h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), RED_SOURCE, 0, h->scal + SC_MISC, st);
      if ((rc = sync_read(h, SC_MISC, 2))) return rc;
      const double sumS = h->hs[SC_MISC], sumS2 = h->hs[SC_MISC + 1];
      if ((rc = pf_solve<double>(h, o, sumS, sumS2, &s.pf_iters))) {
        s.ms_phase_field += now_ms() - tp;
        if (rc == RVE_E_NOCONV) goto fail_out;
        return rc;
      }
      launch_clamp(N, h->rbuf, h->phi_t, h->phi, st);
      launch_fs_stag_norms(N, h->fs_F, h->fs_Fprev, h->fs_Ft, h->phi, h->phi_prev, h->phi_t,
                           h->partial, st);
      launch_reduce(h->partial, voxel_grid(N), 4, 1, h->scal + SC_MISC, st);
      if ((rc = sync_read(h, SC_MISC, 4))) return rc;
      auto ratio = [](double a, double b) { return a == 0.0 ? 0.0 : (b > 0.0 ? a / b : INFINITY); };
      const double re = ratio(h->hs[SC_MISC], h->hs[SC_MISC + 1]);
      const double rp = ratio(h->hs[SC_MISC + 2], h->hs[SC_MISC + 3]);
      HIPCHK(hipMemcpyAsync(h->fs_Fprev, h->fs_F, 9 * N * 8, hipMemcpyDeviceToDevice, st));
      HIPCHK(hipMemcpyAsync(h->phi_prev, h->phi, N * 8, hipMemcpyDeviceToDevice, st));
      s.ms_phase_field += now_ms() - tp;
      if (re <= h->d.tol_stag && rp <= h->d.tol_stag) converged = true;
    }
  }
  if (!converged) { rc = fail(RVE_E_NOCONV, "alternating minimisation reached max_stag"); goto fail_out; }
  {
    int nfail = 0;
    HIPCHK(hipMemcpyAsync(&nfail, h->failc, sizeof(int), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    s.rm_failures = nfail;
    if (nfail > 0) { rc = fail(RVE_E_NOCONV, "return mapping did not converge"); goto fail_out; }
  }
  {   // ---- commit ----
    double tcm = now_ms();
    launch_fs_commit(N, h->fs_P, h->fs_F, h->fs_Fp, h->fs_fptr, h->gslip, h->rho_ssd, h->rho_gnd,
                     h->wp, h->gs, h->H, h->wcrit, h->trig, h->fs_aux, h->phi, m, h->partial, st);
    const int nb = voxel_grid(N);
    launch_reduce(h->partial, nb, 19, 0, h->scal + SC_FM, st);
    launch_reduce(h->partial + 19LL * nb, nb, 2, 1, h->scal + SC_FM + 19, st);
    // GND density of the regularised curl of Fp (the identity has no curl)
    C* B9 = (C*)h->spec;
    o.fwd(h->fs_Fp, true, N, 9, B9);
    launch_curl_reg<double>(h->pl, B9, o.NH, h->d.ell_fp, invN, st);
    o.inv(B9, 9, h->rbuf, true, N, 1.0, 0);
    launch_gnd(N, h->rbuf, h->grain, h->gtab, h->Q81, h->d.burgers, h->rho_gnd, st);
    if (m.flow == FLOW_DUNNE)
      launch_taylor(N, h->gslip, h->rho_ssd, h->rho_gnd, h->grain, h->gtab, m.mu_b, st);
    if ((rc = sync_read(h, SC_FM, 21))) return rc;
    for (int c = 0; c < 9; ++c) {
      s.macro_pk1[c] = h->hs[SC_FM + c] * invN;
      s.macro_defgrad[c] = h->hs[SC_FM + 9 + c] * invN;
    }
    static const int ij[6][2] = {{0, 0}, {1, 1}, {2, 2}, {1, 2}, {0, 2}, {0, 1}};
    for (int c = 0; c < 6; ++c) {
      const int a = 3 * ij[c][0] + ij[c][1], b = 3 * ij[c][1] + ij[c][0];
      s.macro_stress[c] = 0.5 * (s.macro_pk1[a] + s.macro_pk1[b]);
      s.macro_strain[c] = 0.5 * (s.macro_defgrad[a] + s.macro_defgrad[b]) - (c < 3 ? 1.0 : 0.0);
    }
    s.n_triggered = h->hs[SC_FM + 18];
    s.max_phi = h->hs[SC_FM + 19];
    s.max_phi_slip = h->hs[SC_FM + 20];
    s.ms_commit = now_ms() - tcm;
  }
  s.ms_total = now_ms() - t0;
  s.cg_batch = 1;
  if (out) *out = s;
  return RVE_OK;

fail_out:
  {
    std::string msg = g_err;
    (void)hipMemcpyAsync(h->fs_F, h->fs_Ft, 9 * N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(h->sig, h->sig_t, 6 * N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipMemcpyAsync(h->phi, h->phi_t, N * 8, hipMemcpyDeviceToDevice, st);
    (void)hipStreamSynchronize(st);
    s.ms_total = now_ms() - t0;
    if (out) *out = s;
    g_err = msg;
  }
  return rc;
}

int create_impl(rve_s* h, const rve_desc* d, void* dev_arena, size_t arena_bytes,
                void* hip_stream, rve_s** out);
static_assert(SC_N == 544, "rve_s::hs_static holds SC_N host scalars");

}  // namespace

// ---- C ABI -------------------------------------------------------------------------
extern "C" {

const char* rve_last_error(void) { return g_err.c_str(); }

int rve_diag_partials(const rve_desc* d, int64_t* out3) {
  if (!out3) return fail(RVE_E_ARG, "null output");
  const int rc = validate(d);
  if (rc) return rc;
  rve_s tmp;
  tmp.d = *d;
  init_grid(&tmp);
  out3[0] = max_div_partials(tmp.g);
  out3[1] = cg_partial_offset(tmp.g);
  out3[2] = partial_count(tmp.g);
  return RVE_OK;
}

size_t rve_footprint_bytes(const rve_desc* d) {
  if (validate(d) != RVE_OK) return 0;
  rve_s tmp;
  tmp.d = *d;
  init_grid(&tmp);
  tmp.base = nullptr;
  layout(&tmp);
  return tmp.used;
}

int rve_create(const rve_desc* d, void* dev_arena, size_t arena_bytes, void* hip_stream,
               rve_s** out) {
  if (!out) return fail(RVE_E_ARG, "null output handle");
  *out = nullptr;
  int rc = validate(d);
  if (rc) return rc;
  return create_impl(new rve_s(), d, dev_arena, arena_bytes, hip_stream, out);
}

}  // extern "C"

namespace {
// Builds a handle in h (owned by the caller on failure paths of the static variant; the
// heap variant deletes it).  With h->static_dev >= 0 nothing is allocated: the host
// scalars live in the handle and the CG iterations are launched eagerly (a graph
// instantiation allocates).
int create_impl(rve_s* h, const rve_desc* d, void* dev_arena, size_t arena_bytes,
                void* hip_stream, rve_s** out) {
  const bool is_static = h->static_dev >= 0;
  auto drop = [&]() {
    if (!is_static) {
      if (h->hs) (void)hipHostFree(h->hs);
      delete h;
    }
  };
  h->d = *d;
  init_grid(h);
  h->base = nullptr;
  layout(h);
  if (!dev_arena) { drop(); return fail(RVE_E_ARG, "null arena"); }
  if (arena_bytes < h->used) {
    drop();
    return fail(RVE_E_NOMEM, "arena smaller than rve_footprint_bytes");
  }
  h->base = (char*)dev_arena;
  h->cap = arena_bytes;
  layout(h);
  h->st = (hipStream_t)hip_stream;
  (void)hipGetDevice(&h->device);
  crystal_frame(h->d.C11, h->d.C12, h->d.C44, &h->cf);
  fs_frame(h->d.C11, h->d.C12, h->d.C44, &h->ff);
  {
    // CG iterations replay captured graphs on small, launch-bound grids only: at 128^3
    // eager launches measured faster (a replay leaves ~8 us before the next graph's first
    // kernel); RVE_GRAPHS=1 / 0 forces either way
    const char* ev = std::getenv("RVE_GRAPHS");
    const bool small = h->g.nvox <= 64LL * 64 * 64;
    h->use_graphs = (h->st != nullptr) && (ev ? ev[0] == '1' : small) && !is_static;
  }
  if (is_static) {
    h->hs = h->hs_static;
  } else if (hipHostMalloc((void**)&h->hs, SC_N * sizeof(double), hipHostMallocDefault) !=
             hipSuccess) {
    h->hs = nullptr;
    drop();
    return fail(RVE_E_DEVICE, "hipHostMalloc failed");
  }
  // twiddle tables, exp(-2 pi i k / n), computed in FP64
  for (int a = 0; a < 3; ++a) {
    const int n = h->pl.ax[a].n;     // <= 512
    double t64[1024];
    float t32[1024];
    for (int k = 0; k < n; ++k) {
      // reduce the angle to the first octant-friendly form k/n in [0, 1)
      const double ang = -2.0 * M_PI * (double)k / (double)n;
      t64[2 * k] = std::cos(ang);
      t64[2 * k + 1] = std::sin(ang);
      t32[2 * k] = (float)t64[2 * k];
      t32[2 * k + 1] = (float)t64[2 * k + 1];
    }
    // (pageable sources: the copies are staged before hipMemcpyAsync returns; the
    // synchronisation below orders them before any use)
    if (hipMemcpyAsync((void*)h->pl.tw64[a], t64, n * 16, hipMemcpyHostToDevice, h->st) !=
            hipSuccess ||
        hipMemcpyAsync((void*)h->pl.tw32[a], t32, n * 8, hipMemcpyHostToDevice, h->st) !=
            hipSuccess ||
        hipStreamSynchronize(h->st) != hipSuccess) {
      drop();
      return fail(RVE_E_DEVICE, "twiddle upload failed");
    }
  }
  if (upload_reg_twiddles(h->st) != hipSuccess) {
    drop();
    return fail(RVE_E_DEVICE, "register DFT table upload failed");
  }
  double Q[81];
  gnd_q(Q);
  for (int i = 0; i < SC_N; ++i) h->hs[i] = 0.0;
  h->hs[SC_ONE] = 1.0;
  if (hipMemcpyAsync(h->Q81, Q, 81 * 8, hipMemcpyHostToDevice, h->st) != hipSuccess ||
      hipMemcpyAsync(h->scal, h->hs, SC_N * sizeof(double), hipMemcpyHostToDevice, h->st) !=
          hipSuccess ||
      hipStreamSynchronize(h->st) != hipSuccess) {
    drop();
    return fail(RVE_E_DEVICE, "table upload failed");
  }
  *out = h;
  return RVE_OK;
}

// ---- allocation-free handles ----------------------------------------------------------
// One static arena per device for callers that cannot allocate device memory.  In host
// code `scratch` names a host-side stand-in: its device address comes from
// hipGetSymbolAddress, once per device with that device current, and only that address
// is ever handed to the device.
constexpr size_t kScratchBytes = (size_t)320 << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
bool g_scratch_busy[kMaxDevices] = {};
rve_s g_static_handle[kMaxDevices];

}  // namespace

extern "C" {

int rve_create_noalloc(const rve_desc* d, void* hip_stream, rve_s** out) {
  if (!out) return fail(RVE_E_ARG, "null output handle");
  *out = nullptr;
  int rc = validate(d);
  if (rc) return rc;
  {
    rve_s tmp;
    tmp.d = *d;
    init_grid(&tmp);
    tmp.base = nullptr;
    layout(&tmp);
    if (tmp.used > kScratchBytes)
      return fail(RVE_E_NOMEM, "description needs " + std::to_string(tmp.used) +
                                   " device bytes; the static arena holds " +
                                   std::to_string(kScratchBytes));
  }
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return fail(RVE_E_DEVICE, "no current HIP device");
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
      (void)hipGetLastError();
      return fail(RVE_E_DEVICE, "hipGetSymbolAddress of the static arena failed");
    }
    g_scratch_ptr[dev] = p;
  }
  if (g_scratch_busy[dev])
    return fail(RVE_E_STATE, "the device's static arena is held by another handle");
  rve_s* h = &g_static_handle[dev];
  *h = rve_s();
  h->static_dev = dev;
  rc = create_impl(h, d, g_scratch_ptr[dev], kScratchBytes, hip_stream, out);
  if (rc == RVE_OK) g_scratch_busy[dev] = true;
  return rc;
}

int rve_set_microstructure(rve_s* h, const int32_t* grain, int32_t n_grains, const double* quat,
                           const double* tau0, const double* phi0) {
  if (!h || !grain || !quat) return fail(RVE_E_ARG, "null argument");
  if (n_grains < 1 || n_grains > h->d.max_grains) return fail(RVE_E_ARG, "n_grains out of range");
  const long long N = h->g.nvox;
  for (long long v = 0; v < N; ++v)
    if (grain[v] < 0 || grain[v] >= n_grains) return fail(RVE_E_ARG, "grain id out of range");
  std::vector<double> tab((size_t)n_grains * GT_STRIDE);
  for (int gi = 0; gi < n_grains; ++gi) {
    const double* q = quat + 4 * gi;
    const double nq = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    if (!std::isfinite(nq) || std::fabs(nq - 1.0) > 1e-6) return fail(RVE_E_ARG, "quaternion not unit");
    if (tau0 && !(tau0[gi] > 0.0 && std::isfinite(tau0[gi]))) return fail(RVE_E_ARG, "bad tau_c0");
    if (!grain_table(q, h->d.C11, h->d.C12, h->d.C44, tab.data() + (size_t)gi * GT_STRIDE))
      return fail(RVE_E_ARG, "singular stiffness");
    tab[(size_t)gi * GT_STRIDE + GT_TAU0] = tau0 ? tau0[gi] : h->d.tau_c0;
  }
  // initial strength: tau_c0, plus the Taylor term of the initial SSD density
  const double taylor0 =
      h->d.material == RVE_MAT_DUNNE ? h->d.mu * h->d.burgers * std::sqrt(h->d.rho0) : 0.0;
  std::vector<double> g((size_t)N), ph((size_t)N, 0.0), rho((size_t)N, h->d.rho0);
  for (long long v = 0; v < N; ++v) {
    if (phi0) {
      if (!(phi0[v] >= 0.0 && phi0[v] <= 1.0)) return fail(RVE_E_ARG, "phi0 outside [0,1]");
      ph[v] = phi0[v];
    }
    g[v] = (ph[v] >= 1.0) ? INFINITY : (tau0 ? tau0[grain[v]] : h->d.tau_c0) + taylor0;
  }
  h->n_preset = 0;
  for (long long v = 0; v < N; ++v) h->n_preset += ph[v] >= 1.0;
  hipStream_t st = h->st;
  HIPCHK(hipMemcpyAsync(h->gtab, tab.data(), tab.size() * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->grain, grain, N * 4, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->gslip, g.data(), N * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->phi, ph.data(), N * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->rho_ssd, rho.data(), N * 8, hipMemcpyHostToDevice, st));
  double* zero6[] = {h->eps, h->sig, h->epsp};
  for (double* p : zero6) launch_zero(p, 6 * N * 8, st);
  launch_zero(h->beta, 9 * N * 8, st);
  double* zero1[] = {h->rho_gnd, h->wp, h->gs, h->H, h->wcrit, h->trig, h->S, h->wep};
  for (double* p : zero1) launch_zero(p, N * 8, st);
  if (h->fs) {      // F = Fp = I, no stress
    const double I9[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1};
    for (double* p : {h->fs_F, h->fs_Fp}) {
      launch_zero(p, 9 * N * 8, st);
      launch_fs_add_uniform(N, p, I9, st);
    }
    launch_zero(h->fs_P, 9 * N * 8, st);
  }
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  for (int c = 0; c < 6; ++c) h->msig_t[c] = h->meps_t[c] = 0.0;
  h->micro = true;
  h->n_grains = n_grains;
  return RVE_OK;
}

int rve_step_increment_mixed(rve_s* h, const double deps[6], const double dsig[6],
                             int32_t stress_mask, double dt, rve_stats* st) {
  if (!h || !deps) return fail(RVE_E_ARG, "null argument");
  if (!h->micro) return fail(RVE_E_STATE, "microstructure not set");
  if (h->fs) return fail(RVE_E_ARG, "finite-strain handle: use rve_step_increment_finite");
  if (stress_mask < 0 || stress_mask > 63) return fail(RVE_E_ARG, "stress_mask outside 0..63");
  if (stress_mask && !dsig) return fail(RVE_E_ARG, "null stress increment");
  if (h->d.plane_stress && ((stress_mask & 0b011100) || deps[2] != 0.0 || deps[3] != 0.0 ||
                            deps[4] != 0.0))
    return fail(RVE_E_ARG, "plane stress: the out-of-plane components (zz, yz, xz) are "
                           "stress free at every voxel and take no macro control");
  double ds[6] = {0, 0, 0, 0, 0, 0};
  for (int c = 0; c < 6; ++c) {
    const bool f = (stress_mask >> c) & 1;
    if (f) ds[c] = dsig[c];
    if (!std::isfinite(f ? ds[c] : deps[c])) return fail(RVE_E_ARG, "non-finite macro increment");
  }
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RVE_E_ARG, "dt must be positive and finite");
  g_err.clear();
  int cur = -1;
  if (hipGetDevice(&cur) == hipSuccess && cur != h->device) HIPCHK(hipSetDevice(h->device));
  return h->f64 ? run_increment<double>(h, deps, ds, stress_mask, dt, st)
                : run_increment<float>(h, deps, ds, stress_mask, dt, st);
}

int rve_step_increment_finite(rve_s* h, const double dF[9], double dt, rve_stats* st) {
  if (!h || !dF) return fail(RVE_E_ARG, "null argument");
  if (!h->fs) return fail(RVE_E_ARG, "small-strain handle: use rve_step_increment");
  if (!h->micro) return fail(RVE_E_STATE, "microstructure not set");
  for (int c = 0; c < 9; ++c)
    if (!std::isfinite(dF[c])) return fail(RVE_E_ARG, "non-finite increment");
  if (!(dt > 0.0) || !std::isfinite(dt)) return fail(RVE_E_ARG, "dt must be positive");
  g_err.clear();
  return run_increment_fs(h, dF, dt, st);
}

int rve_step_increment(rve_s* h, const double deps[6], double dt, rve_stats* st) {
  return rve_step_increment_mixed(h, deps, nullptr, 0, dt, st);
}

int rve_pool_step(rve_s* const* hs, int32_t n, const double* deps, const double* dt,
                  int32_t* status, rve_stats* stats) {
  if (n < 0 || (n > 0 && (!hs || !deps || !dt || !status))) return fail(RVE_E_ARG, "bad argument");
  for (int i = 0; i < n; ++i)
    for (int j = i + 1; j < n; ++j)
      if (hs[i] == hs[j]) return fail(RVE_E_ARG, "handles must be distinct");
  for (int i = 0; i < n; ++i)
    if (!hs[i]) return fail(RVE_E_ARG, "null handle");
  // groups of handles that can share CG launches: same grid, voxel size, precision,
  // derivative and CG solver on one device, small-strain kinematics, fused z passes, and the
  // same arena layout (the batched launches find every handle's buffers at the leader's
  // offsets, so every option that places buffers must agree)
  std::vector<std::unique_ptr<CgGroup>> groups;
  std::vector<CgGroup*> gof((size_t)n, nullptr);
  auto same = [](const rve_s* a, const rve_s* b) {
    return a->d.n[0] == b->d.n[0] && a->d.n[1] == b->d.n[1] && a->d.n[2] == b->d.n[2] &&
           a->d.h == b->d.h && a->d.precision == b->d.precision && a->d.deriv == b->d.deriv &&
           a->device == b->device && a->d.max_krylov == b->d.max_krylov &&
           a->d.max_grains == b->d.max_grains && a->d.gnd_coupling == b->d.gnd_coupling &&
           a->d.plane_stress == b->d.plane_stress && a->d.krylov == b->d.krylov &&
           a->used == b->used;
  };
  auto can_batch = [](const rve_s* a) {
    return !a->fs && a->d.krylov == RVE_KRYLOV_CG && a->time_xt == 0 &&
           (a->f64 ? fused_z_available<double>(a->pl) : fused_z_available<float>(a->pl));
  };
  if (!pool_batching_off()) {
    for (int i = 0; i < n; ++i) {
      if (!can_batch(hs[i]) || gof[i]) continue;
      int cnt = 0;
      for (int j = i; j < n; ++j) cnt += can_batch(hs[j]) && !gof[j] && same(hs[i], hs[j]);
      if (cnt < 2) continue;
      groups.emplace_back(new CgGroup());
      CgGroup* G = groups.back().get();
      for (int j = i; j < n && G->members < kMaxBatch; ++j)
        if (can_batch(hs[j]) && !gof[j] && same(hs[i], hs[j])) {
          gof[j] = G;
          G->members++;
        }
    }
  }
  std::vector<std::string> errs((size_t)n);
  auto one = [&](int i) {
    hs[i]->cg_group = gof[i];
    status[i] = rve_step_increment(hs[i], deps + 6 * i, dt[i], stats ? stats + i : nullptr);
    if (status[i] != RVE_OK) errs[i] = g_err;
    hs[i]->cg_group = nullptr;
    if (CgGroup* G = gof[i]) {       // no leader waits for a handle that has finished
      std::lock_guard<std::mutex> lk(G->mu);
      G->members--;
      G->cv.notify_all();
    }
  };
  if (n == 1) {
    one(0);
  } else {
    std::vector<std::thread> th;
    th.reserve((size_t)n);
    for (int i = 0; i < n; ++i) th.emplace_back(one, i);
    for (auto& t : th) t.join();
  }
  for (int i = 0; i < n; ++i)
    if (status[i] != RVE_OK) return fail(status[i], "handle " + std::to_string(i) + ": " + errs[i]);
  return RVE_OK;
}

static const uint32_t kSmallOnly =
    RVE_F_STRAIN | RVE_F_STRESS | RVE_F_STRESS_EFF | RVE_F_EPS_P | RVE_F_BETA_P;
static const uint32_t kFiniteOnly = RVE_F_DEFGRAD | RVE_F_PK1 | RVE_F_FP;

size_t rve_fields_count(const rve_s* h, uint32_t mask) {
  if (!h) return 0;
  if (mask >> 17) return 0;
  if (mask & (h->fs ? kSmallOnly : kFiniteOnly)) return 0;
  const uint32_t six = RVE_F_STRAIN | RVE_F_STRESS | RVE_F_STRESS_EFF | RVE_F_EPS_P;
  const uint32_t nine = RVE_F_BETA_P | kFiniteOnly;
  size_t c = 0;
  for (int b = 0; b < 17; ++b) {
    const uint32_t bit = 1u << b;
    if (!(mask & bit)) continue;
    c += (bit & six) ? 6 : ((bit & nine) ? 9 : 1);
  }
  return c * (size_t)h->g.nvox;
}

int rve_fields(rve_s* h, uint32_t mask, double* out, size_t n) {
  if (!h || !out) return fail(RVE_E_ARG, "null argument");
  if (!h->micro) return fail(RVE_E_STATE, "microstructure not set");
  if (mask >> 17) return fail(RVE_E_ARG, "unknown field bit");
  if (mask & (h->fs ? kSmallOnly : kFiniteOnly))
    return fail(RVE_E_ARG, h->fs ? "small-strain field of a finite-strain handle"
                                 : "finite-strain field of a small-strain handle");
  const size_t need = rve_fields_count(h, mask);
  if (n < need) return fail(RVE_E_ARG, "output buffer too small");
  const long long N = h->g.nvox;
  hipStream_t st = h->st;
  double* o = out;
  auto cp = [&](const double* src, int nc) -> int {
    HIPCHK(hipMemcpyAsync(o, src, (size_t)nc * N * 8, hipMemcpyDeviceToHost, st));
    o += (size_t)nc * N;
    return RVE_OK;
  };
  int rc = RVE_OK;
  for (int b = 0; b < 17 && rc == RVE_OK; ++b) {
    const uint32_t bit = 1u << b;
    if (!(mask & bit)) continue;
    switch (bit) {
      case RVE_F_STRAIN: rc = cp(h->eps, 6); break;
      case RVE_F_STRESS:      // degraded on the device into the phase-field scratch
        launch_degrade(N, h->sig, h->phi, h->d.k_res, h->rbuf, st);
        rc = cp(h->rbuf, 6);
        break;
      case RVE_F_STRESS_EFF: rc = cp(h->sig, 6); break;
      case RVE_F_DAMAGE: rc = cp(h->phi, 1); break;
      case RVE_F_GS: rc = cp(h->gs, 1); break;
      case RVE_F_RHO_SSD: rc = cp(h->rho_ssd, 1); break;
      case RVE_F_RHO_GND: rc = cp(h->rho_gnd, 1); break;
      case RVE_F_WP: rc = cp(h->wp, 1); break;
      case RVE_F_H: rc = cp(h->H, 1); break;
      case RVE_F_WCRIT: rc = cp(h->wcrit, 1); break;
      case RVE_F_TRIG: rc = cp(h->trig, 1); break;
      case RVE_F_EPS_P: rc = cp(h->epsp, 6); break;
      case RVE_F_SLIP_RES: rc = cp(h->gslip, 1); break;
      case RVE_F_BETA_P: rc = cp(h->beta, 9); break;
      case RVE_F_DEFGRAD: rc = cp(h->fs_F, 9); break;
      case RVE_F_PK1:         // degraded on the device into the phase-field scratch
        launch_fs_degrade(N, h->fs_P, h->phi, h->d.k_res, h->rbuf, st);
        rc = cp(h->rbuf, 9);
        break;
      case RVE_F_FP: rc = cp(h->fs_Fp, 9); break;
    }
  }
  if (rc) return rc;
  HIPCHK(hipStreamSynchronize(st));
  return RVE_OK;
}

}  // extern "C"
namespace {
void pool_release(rve_pool_s* p, size_t off, size_t len);
}
extern "C" {

int rve_destroy(rve_s* h) {
  if (!h) return RVE_OK;
  if (h->st) (void)hipStreamSynchronize(h->st);
  else (void)hipDeviceSynchronize();
  for (hipGraphExec_t& e : h->cg_exec)
    if (e) (void)hipGraphExecDestroy(e);
  for (hipEvent_t e : h->xt_ev) (void)hipEventDestroy(e);
  if (h->cg_ready) (void)hipEventDestroy(h->cg_ready);
  if (h->cg_done) (void)hipEventDestroy(h->cg_done);
  h->cg_ready = h->cg_done = nullptr;
  if (h->static_dev >= 0) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    g_scratch_busy[h->static_dev] = false;
    h->xt_ev.clear();
    h->hs = nullptr;
    return RVE_OK;
  }
  if (h->hs) (void)hipHostFree(h->hs);
  rve_pool_s* pool = h->pool;
  const size_t off = h->pool_off, len = h->pool_len;
  delete h;
  if (pool) pool_release(pool, off, len);
  return RVE_OK;
}

}  // extern "C"

// ---- diagnostics -------------------------------------------------------------------
template <typename R>
static int diag_pass(rve_s* h, int pass_id, int reps, double* bytes) {
  typedef cplx<R> C;
  Ops<R> o(h);
  const double N = (double)h->g.nvox, NH = (double)h->g.nspec;
  const double cb = sizeof(C), rb = sizeof(R);
  double b = 0.0;
  hipStream_t st = h->st;
  for (int k = 0; k < reps; ++k) {
    switch (pass_id) {
      case RVE_PASS_FFT_Z: launch_fft_yz<R>(h->pl, o.W, h->g.nspec, 6, 2, true, st); break;
      case RVE_PASS_FFT_Y: launch_fft_yz<R>(h->pl, o.W, h->g.nspec, 6, 1, true, st); break;
      case RVE_PASS_X_TANGENT: launch_x_tangent<R>(h->pl, o.W, h->g.nspec, o.gK(), 1.0 / N, st); break;
      case RVE_PASS_GRAD: launch_sym_grad<R>(h->pl, o.v(3), h->g.nspec, o.W, h->g.nspec, st); break;
      case RVE_PASS_DIV: launch_div<R>(h->pl, o.W, h->g.nspec, o.v(4), h->g.nspec, -1.0, st); break;
      case RVE_PASS_PRECOND:
        launch_precond<R>(h->pl, o.v(1), o.v(2), h->g.nspec, h->scal + SC_KBAR, h->partial, st);
        break;
      case RVE_PASS_CONSTITUTIVE: o.cur_dt = 1.0; o.constitutive(nullptr, 0.0, h->phi); break;
      case RVE_PASS_MATVEC: o.matvec(o.v(3), o.v(4), o.v(5)); break;
      case RVE_PASS_ZGRAD:
        launch_zgrad_inv<R>(h->pl, o.v(2), o.v(3), o.v(5), h->g.nspec, h->scal, SC_ONE, SC_ONE,
                            o.W, st);
        break;
      case RVE_PASS_ZDIV:
        launch_zdiv_fwd<R>(h->pl, o.W, o.v(4), o.v(3), h->g.nspec, h->partial, st);
        break;
      case RVE_PASS_PF_ITER: {   // the launches of one phase-field CG iteration (pf_solve)
        const long long n = h->g.nvox;
        double *X = h->rbuf, *Rr = h->rbuf + n, *Z = h->rbuf + 2 * n, *P = h->rbuf + 3 * n,
               *Wv = h->rbuf + 4 * n;
        double* sc = h->scal;
        C* W1 = (C*)h->spec;
        int nb = launch_pf_pq(n, P, Wv, h->S, h->partial, st);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_PQ, st);
        nb = launch_pf_xr(n, X, Rr, P, Wv, h->S, sc, SC_RZ0, SC_PQ, h->partial, st);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_RR, st);
        launch_pf_check(sc, SC_FLAG, SC_ITER, SC_PQ, SC_RR, SC_TOL2, st);
        launch_x_r2c<R>(h->pl, Rr, true, n, nullptr, 0.0, W1, o.NH, 1, st);
        launch_fft_yz<R>(h->pl, W1, o.NH, 1, 1, false, st);
        launch_fft_yz<R>(h->pl, W1, o.NH, 1, 2, false, st);
        launch_pf_scale<R>(h->pl, W1, h->d.ell, 1.0 / N, st);
        launch_fft_yz<R>(h->pl, W1, o.NH, 1, 2, true, st);
        launch_fft_yz<R>(h->pl, W1, o.NH, 1, 1, true, st);
        launch_x_c2r<R>(h->pl, W1, o.NH, Z, true, n, 1, 1.0, 0, st);
        nb = launch_rdot(n, Rr, Z, h->partial, st);
        launch_reduce(h->partial, nb, 1, 0, sc + SC_RZ1, st);
        launch_pf_pw(n, P, Wv, Z, Rr, sc, SC_RZ1, SC_RZ0, st);
        break;
      }
    }
  }
  switch (pass_id) {
    case RVE_PASS_FFT_Z: case RVE_PASS_FFT_Y: b = 2 * 6 * NH * cb; break;
    case RVE_PASS_X_TANGENT: b = 2 * 6 * NH * cb + 21 * N * rb; break;
    case RVE_PASS_GRAD: case RVE_PASS_DIV: b = 9 * NH * cb; break;
    case RVE_PASS_PRECOND: b = 6 * NH * cb; break;
    case RVE_PASS_CONSTITUTIVE: b = N * (4 * 6 * 8 + 3 * 8 + 4 + 6 * 8 + 21 * rb); break;
    case RVE_PASS_MATVEC:
      b = (fused_z_available<R>(h->pl) ? 5 * 12 : 9 + 4 * 12 + 12 + 9) * NH * cb + 21 * N * rb;
      break;
    case RVE_PASS_ZGRAD: b = 15 * NH * cb; break;
    case RVE_PASS_ZDIV: b = 12 * NH * cb; break;
    // FP64 vectors: pf_pq 3, pf_xr 7, rdot 2, pf_pw 6 and the real ends of the FFT round trip
    // 2 reals per voxel; the one-component FFT round trip 12 half-spectrum values
    case RVE_PASS_PF_ITER: b = 20 * N * 8 + 12 * NH * cb; break;
  }
  if (bytes) *bytes = b;
  HIPCHK(hipGetLastError());
  return RVE_OK;
}

template <typename R>
static int diag_fft(rve_s* h, int ncomp, const double* in, double* out, bool forward) {
  typedef cplx<R> C;
  Ops<R> o(h);
  const long long N = h->g.nvox, NH = h->g.nspec;
  C* W = (C*)h->spec;
  hipStream_t st = h->st;
  if (forward) {
    HIPCHK(hipMemcpyAsync(h->rbuf, in, (size_t)ncomp * N * 8, hipMemcpyHostToDevice, st));
    o.fwd(h->rbuf, true, N, ncomp, W);
    std::vector<C> tmp((size_t)ncomp * NH);
    HIPCHK(hipMemcpyAsync(tmp.data(), W, tmp.size() * sizeof(C), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < tmp.size(); ++i) { out[2 * i] = tmp[i].x; out[2 * i + 1] = tmp[i].y; }
  } else {
    std::vector<C> tmp((size_t)ncomp * NH);
    for (size_t i = 0; i < tmp.size(); ++i) { tmp[i].x = (R)in[2 * i]; tmp[i].y = (R)in[2 * i + 1]; }
    HIPCHK(hipMemcpyAsync(W, tmp.data(), tmp.size() * sizeof(C), hipMemcpyHostToDevice, st));
    o.inv(W, ncomp, h->rbuf, true, N, 1.0 / (double)N, 0);
    HIPCHK(hipMemcpyAsync(out, h->rbuf, (size_t)ncomp * N * 8, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  HIPCHK(hipGetLastError());
  return RVE_OK;
}

template <typename R>
static int diag_const(rve_s* h, const double* eps6, double dt, double* sig_out, double* gk_out) {
  Ops<R> o(h);
  o.cur_dt = dt;
  const long long N = h->g.nvox;
  hipStream_t st = h->st;
  // keep the state: eps -> eps_prev, sig -> sig_t (restored below)
  HIPCHK(hipMemcpyAsync(h->eps_prev, h->eps, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->sig_t, h->sig, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->eps, eps6, 6 * N * 8, hipMemcpyHostToDevice, st));
  launch_zero(h->failc, sizeof(int), st);
  o.constitutive(nullptr, 0.0, h->phi);
  o.kbar();
  if (sig_out) HIPCHK(hipMemcpyAsync(sig_out, h->sig, 6 * N * 8, hipMemcpyDeviceToHost, st));
  if (gk_out) {
    std::vector<R> tmp((size_t)21 * N);
    HIPCHK(hipMemcpyAsync(tmp.data(), h->gK, tmp.size() * sizeof(R), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    for (size_t i = 0; i < tmp.size(); ++i) gk_out[i] = (double)tmp[i];
  }
  int nfail = 0;
  HIPCHK(hipMemcpyAsync(&nfail, h->failc, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipMemcpyAsync(h->eps, h->eps_prev, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipMemcpyAsync(h->sig, h->sig_t, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  if (nfail) return fail(RVE_E_NOCONV, "return mapping did not converge");
  return RVE_OK;
}

template <typename R>
static int diag_op(rve_s* h, const double* u3, double* v3) {
  typedef cplx<R> C;
  Ops<R> o(h);
  const long long N = h->g.nvox, NH = h->g.nspec;
  hipStream_t st = h->st;
  HIPCHK(hipMemcpyAsync(h->rbuf, u3, 3 * N * 8, hipMemcpyHostToDevice, st));
  o.fwd(h->rbuf, true, N, 3, o.v(3));
  o.matvec(o.v(3), o.v(4), o.v(5));
  launch_precond<R>(h->pl, o.v(4), o.v(2), NH, h->scal + SC_KBAR, h->partial, st);
  HIPCHK(hipMemcpyAsync(o.W, o.v(2), 3 * NH * sizeof(C), hipMemcpyDeviceToDevice, st));
  o.inv(o.W, 3, h->rbuf, true, N, 1.0 / (double)N, 0);
  HIPCHK(hipMemcpyAsync(v3, h->rbuf, 3 * N * 8, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  return RVE_OK;
}

extern "C" {

int rve_diag_pass(rve_s* h, int32_t pass_id, int32_t reps, double* bytes) {
  if (h && h->fs) return fail(RVE_E_ARG, "finite-strain handle (see rve_diag_constitutive_finite)");
  if (!h || reps < 0 || pass_id < 0 || pass_id > RVE_PASS_PF_ITER) return fail(RVE_E_ARG, "bad argument");
  if ((pass_id == RVE_PASS_ZGRAD || pass_id == RVE_PASS_ZDIV) &&
      !(h->f64 ? fused_z_available<double>(h->pl) : fused_z_available<float>(h->pl)))
    return fail(RVE_E_ARG, "no fused z pass for this grid");
  if (pass_id == RVE_PASS_CONSTITUTIVE && !h->micro) return fail(RVE_E_STATE, "microstructure not set");
  return h->f64 ? diag_pass<double>(h, pass_id, reps, bytes) : diag_pass<float>(h, pass_id, reps, bytes);
}

int rve_diag_time_pass(rve_s* h, int32_t pass_id, int32_t on) {
  if (!h || pass_id != RVE_PASS_X_TANGENT) return fail(RVE_E_ARG, "only RVE_PASS_X_TANGENT is timed live");
  if (on < 0) return fail(RVE_E_ARG, "negative timing period");
  h->time_xt = on;
  h->xt_used = 0;
  return RVE_OK;
}

int rve_diag_pass_time(rve_s* h, int64_t* launches, double* total_ms) {
  if (!h || !launches || !total_ms) return fail(RVE_E_ARG, "null argument");
  *launches = h->xt_launches;
  *total_ms = h->xt_ms;
  h->xt_launches = 0;
  h->xt_ms = 0.0;
  return RVE_OK;
}

int rve_diag_rfft(rve_s* h, int32_t ncomp, const double* in, double* out) {
  if (!h || !in || !out || ncomp < 1 || ncomp > 9) return fail(RVE_E_ARG, "bad argument");
  return h->f64 ? diag_fft<double>(h, ncomp, in, out, true) : diag_fft<float>(h, ncomp, in, out, true);
}

int rve_diag_irfft(rve_s* h, int32_t ncomp, const double* in, double* out) {
  if (!h || !in || !out || ncomp < 1 || ncomp > 9) return fail(RVE_E_ARG, "bad argument");
  return h->f64 ? diag_fft<double>(h, ncomp, in, out, false)
                : diag_fft<float>(h, ncomp, in, out, false);
}

int rve_diag_constitutive(rve_s* h, const double* eps6, double dt, double* sig6, double* gk21) {
  if (h && h->fs) return fail(RVE_E_ARG, "finite-strain handle (see rve_diag_constitutive_finite)");
  if (!h || !eps6 || !(dt > 0.0)) return fail(RVE_E_ARG, "bad argument");
  if (!h->micro) return fail(RVE_E_STATE, "microstructure not set");
  return h->f64 ? diag_const<double>(h, eps6, dt, sig6, gk21)
                : diag_const<float>(h, eps6, dt, sig6, gk21);
}

int rve_diag_constitutive_finite(rve_s* h, const double* F9, double dt, double* P9,
                                 double* K81) {
  if (!h || !F9) return fail(RVE_E_ARG, "bad argument");
  if (!h->fs) return fail(RVE_E_ARG, "small-strain handle");
  if (!h->micro) return fail(RVE_E_STATE, "microstructure not set");
  const long long N = h->g.nvox;
  hipStream_t st = h->st;
  Ops<double> o(h);
  const Material m = o.mat(dt);
  // scratch: the input in the Newton correction buffer, the warm starts copied aside,
  // P in the phase-field scratch
  HIPCHK(hipMemcpyAsync(h->fs_dF, F9, 9 * N * 8, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(h->sig_t, h->sig, 6 * N * 8, hipMemcpyDeviceToDevice, st));
  launch_zero(h->failc, sizeof(int), st);
  launch_fs_constitutive(N, h->fs_dF, nullptr, 0.0, h->fs_Fp, h->gslip, h->grain, h->gtab,
                         h->sig_t, h->phi, h->rbuf, h->fs_fptr, h->fs_aux, (double*)h->gK, h->ff,
                         m, h->failc, st);
  if (P9) HIPCHK(hipMemcpyAsync(P9, h->rbuf, 9 * N * 8, hipMemcpyDeviceToHost, st));
  if (K81) HIPCHK(hipMemcpyAsync(K81, h->gK, 81 * N * 8, hipMemcpyDeviceToHost, st));
  int nfail = 0;
  HIPCHK(hipMemcpyAsync(&nfail, h->failc, sizeof(int), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  HIPCHK(hipGetLastError());
  if (nfail) return fail(RVE_E_NOCONV, "return mapping did not converge");
  return RVE_OK;
}

int rve_diag_operator(rve_s* h, const double* u3, double* v3) {
  if (h && h->fs) return fail(RVE_E_ARG, "finite-strain handle (see rve_diag_constitutive_finite)");
  if (!h || !u3 || !v3) return fail(RVE_E_ARG, "bad argument");
  if (!h->micro) return fail(RVE_E_STATE, "microstructure not set");
  return h->f64 ? diag_op<double>(h, u3, v3) : diag_op<float>(h, u3, v3);
}

}  // extern "C"

// ---- radix schedule ------------------------------------------------------------------
namespace rvefft {
bool make_axis_plan(int n, AxisPlan* out) {
  AxisPlan p;
  p.n = n;
  p.nst = 0;
  int m = n;
  while (m % 4 == 0 && p.nst < kMaxStages) { p.radix[p.nst++] = 4; m /= 4; }
  while (m % 2 == 0 && p.nst < kMaxStages) { p.radix[p.nst++] = 2; m /= 2; }
  while (m % 3 == 0 && p.nst < kMaxStages) { p.radix[p.nst++] = 3; m /= 3; }
  for (int i = p.nst; i < kMaxStages; ++i) p.radix[i] = 1;
  *out = p;
  return m == 1;
}
}  // namespace rvefft

// ---- serving pool: one caller-owned device arena shared by many handles -------------
// First fit over the free ranges of the arena (256-byte granules); a handle created in the
// pool takes its footprint from it and gives it back at rve_destroy, where neighbouring
// free ranges merge again.
struct rve_pool_s {
  char* base = nullptr;
  size_t bytes = 0;
  std::mutex mu;
  std::map<size_t, size_t> free_;   // offset -> length of each free range
  int live = 0;
};

namespace {
void pool_release(rve_pool_s* p, size_t off, size_t len) {
  std::lock_guard<std::mutex> lk(p->mu);
  auto next = p->free_.lower_bound(off);
  if (next != p->free_.end() && off + len == next->first) {
    len += next->second;
    next = p->free_.erase(next);
  }
  if (next != p->free_.begin()) {
    auto prev = std::prev(next);
    if (prev->first + prev->second == off) {
      prev->second += len;
      --p->live;
      return;
    }
  }
  p->free_[off] = len;
  --p->live;
}
}  // namespace

extern "C" {

int rve_pool_create(void* dev_arena, size_t arena_bytes, rve_pool_s** out) {
  if (!out) return fail(RVE_E_ARG, "null output");
  *out = nullptr;
  if (!dev_arena) return fail(RVE_E_ARG, "null arena");
  const uintptr_t b = (uintptr_t)dev_arena, a = (b + 255) & ~(uintptr_t)255;
  if (arena_bytes < (a - b) + 256) return fail(RVE_E_ARG, "arena smaller than one granule");
  const size_t len = (arena_bytes - (a - b)) & ~(size_t)255;
  rve_pool_s* p = new (std::nothrow) rve_pool_s;
  if (!p) return fail(RVE_E_NOMEM, "host allocation failed");
  p->base = (char*)a;
  p->bytes = len;
  p->free_[0] = len;
  *out = p;
  return RVE_OK;
}

int rve_create_in_pool(rve_pool_s* pool, const rve_desc* d, void* hip_stream, rve_s** out) {
  if (!pool || !out) return fail(RVE_E_ARG, "null pool or output");
  *out = nullptr;
  const int rc0 = validate(d);
  if (rc0) return rc0;
  const size_t need = align_up(rve_footprint_bytes(d));
  size_t off = 0;
  bool found = false;
  size_t largest = 0;
  {
    std::lock_guard<std::mutex> lk(pool->mu);
    for (auto it = pool->free_.begin(); it != pool->free_.end(); ++it) {
      largest = std::max(largest, it->second);
      if (it->second >= need) {
        off = it->first;
        const size_t rest = it->second - need;
        pool->free_.erase(it);
        if (rest) pool->free_[off + need] = rest;
        found = true;
        ++pool->live;
        break;
      }
    }
  }
  if (!found)
    return fail(RVE_E_NOMEM, "no free range of " + std::to_string(need) +
                                 " bytes in the pool (largest " + std::to_string(largest) + ")");
  const int rc = rve_create(d, pool->base + off, need, hip_stream, out);
  if (rc) {
    pool_release(pool, off, need);
    return rc;
  }
  (*out)->pool = pool;
  (*out)->pool_off = off;
  (*out)->pool_len = need;
  return RVE_OK;
}

size_t rve_pool_free_bytes(rve_pool_s* pool, size_t* largest_range) {
  if (largest_range) *largest_range = 0;
  if (!pool) return 0;
  std::lock_guard<std::mutex> lk(pool->mu);
  size_t tot = 0;
  for (const auto& r : pool->free_) {
    tot += r.second;
    if (largest_range) *largest_range = std::max(*largest_range, r.second);
  }
  return tot;
}

int rve_pool_destroy(rve_pool_s* pool) {
  if (!pool) return RVE_OK;
  {
    std::lock_guard<std::mutex> lk(pool->mu);
    if (pool->live)
      return fail(RVE_E_STATE, std::to_string(pool->live) + " handles of the pool are alive");
  }
  delete pool;
  return RVE_OK;
}

}  // extern "C"
