// z passes fused with the pointwise operators at the two ends of the momentum
// operator (Sec. 3.1, eqs. fdef and momentum): the inverse pass forms the strain
// spectrum sym(i xi~ (x) p) of the updated CG direction while it loads, the forward
// pass contracts the stress spectrum with -i xi~ while it stores, so neither spectrum
// makes an extra trip through HBM.  A work unit is a tile of x-bins at one ky; each
// block takes one component of one unit.  When the units come in multiples of 8, the
// blocks of one unit are numbered 8 apart, so they are dispatched to the same XCD one
// after the other and meet the operands they share in its L2; each XCD takes a contiguous
// range of units, so that the tiles of one row (whose segments share the 128-B lines at
// the tile boundaries: rows of N1/2 + 1 bins do not start on a line) meet there too.
#include "passutil.h"

namespace rvefft {

__device__ __forceinline__ void unit_comp(int nunits, int ncomp, int& u, int& c) {
  const int bid = blockIdx.x;
  if ((nunits & 7) == 0) {
    const int x = bid & 7, s = bid >> 3;
    c = s % ncomp;
    u = x * (nunits >> 3) + s / ncomp;
  } else {
    c = bid % ncomp;
    u = bid / ncomp;
  }
}

// i s a for real s
template <typename R>
__device__ __forceinline__ cplx<R> imul(R s, cplx<R> a) { return cplx<R>{-s * a.y, s * a.x}; }

// Split N = Na x Nb of the fused z passes: a short first pass, so that the several
// operands each first-pass item loads stay in registers together.
template <int N> struct ZSplit;
template <> struct ZSplit<16> { static constexpr int Na = 4, Nb = 4; };
template <> struct ZSplit<32> { static constexpr int Na = 4, Nb = 8; };
template <> struct ZSplit<48> { static constexpr int Na = 3, Nb = 16; };
template <> struct ZSplit<64> { static constexpr int Na = 8, Nb = 8; };
template <> struct ZSplit<96> { static constexpr int Na = 6, Nb = 16; };
template <> struct ZSplit<128> { static constexpr int Na = 8, Nb = 16; };
template <> struct ZSplit<256> { static constexpr int Na = 16, Nb = 16; };

// Rotated-scheme factors of the block's x columns (with its ky) and of every kz, in LDS:
// k_x = Pxy[0][x] Az[kz], k_y = Pxy[1][x] Az[kz], k_z = Pxy[2][x] Dz[kz], with
// Pxy = (Dx Ay, Ax Dy, Ax Ay) (rot_factors).
template <typename R, int N, int P, int NT>
__device__ __forceinline__ void z_rot(const Grid& g, int kx0, int tile, int TX, int ky,
                                      cplx<R>* pxy, cplx<R>* dz, cplx<R>* az) {
  for (int t = threadIdx.x; t < N; t += NT) {
    cplx<double> D, A;
    rot_factors(t, g.n3, g.h, D, A);
    dz[t] = cplx<R>{(R)D.x, (R)D.y};
    az[t] = cplx<R>{(R)A.x, (R)A.y};
  }
  cplx<double> Dy, Ay;
  rot_factors(ky, g.n2, g.h, Dy, Ay);
  for (int t = threadIdx.x; t < P; t += NT) {
    const int cx = (t < TX) ? kx0 + t : (tile == 0 ? g.n1 / 2 : -1);
    cplx<double> Dx{0.0, 0.0}, Ax{0.0, 0.0};
    if (cx >= 0) rot_factors(cx, g.n1, g.h, Dx, Ax);
    const cplx<double> f[3] = {cmul(Dx, Ay), cmul(Ax, Dy), cmul(Ax, Ay)};
    for (int a = 0; a < 3; ++a) pxy[a * P + t] = cplx<R>{(R)f[a].x, (R)f[a].y};
  }
}

// xi~ of the block's x columns, its ky and every kz, in LDS (no divisions in the loops)
template <typename R, int N, int P, int NT>
__device__ __forceinline__ void z_freqs(const Grid& g, int kx0, int tile, int TX, int ky,
                                        R* txs, R* tzs, R& ty) {
  for (int t = threadIdx.x; t < N; t += NT) tzs[t] = (R)freq(t, g.n3, g.L3, true);
  for (int t = threadIdx.x; t < P; t += NT) {
    const int cx = (t < TX) ? kx0 + t : (tile == 0 ? g.n1 / 2 : -1);
    txs[t] = cx >= 0 ? (R)freq(cx, g.n1, g.L1, true) : R(0);
  }
  ty = (R)freq(ky, g.n2, g.L2, true);
}

// p_new = z + (sc[ia]/sc[ib]) p_old, then component c of e = sym(i xi~ (x) p_new) and its
// inverse DFT along z.  The blocks of the diagonal components store p_new.
template <typename R, int N, int TX, int NT, int SCH>
__global__ void __launch_bounds__(NT)
k_zgrad_inv(const cplx<R>* __restrict__ zv, const cplx<R>* __restrict__ pold,
            cplx<R>* __restrict__ pnew, long long cs, double* __restrict__ sc, int ia, int ib,
            cplx<R>* __restrict__ e, Grid g, const cplx<R>* __restrict__ tw_g,
            const double* __restrict__ stop, CgCheck ck) {
  {
    const long long d = slot_delta(g);
    zv = at_slot(zv, d); pold = at_slot(pold, d); pnew = at_slot(pnew, d); sc = at_slot(sc, d);
    e = at_slot(e, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
    ck.part = at_slot(ck.part, d);
  }
  if (stop && *stop != 0.0) return;
  __shared__ double red[2 * (NT / 64)];
  double be;
  if (ck.part) {
    double rz;
    if (cg_check_inline(ck, sc, red, rz)) return;
    be = rz / sc[ib];
  } else {
    be = sc[ia] / sc[ib];
  }
  constexpr int P = TX + 1;                       // the Nyquist column rides in tile 0
  constexpr int Na = ZSplit<N>::Na, Nb = ZSplit<N>::Nb;
  constexpr int PITCH = N + 1;
  __shared__ cplx<R> A[P * PITCH];
  __shared__ cplx<R> tw[N];
  __shared__ R tzs[SCH ? 1 : N], txs[SCH ? 1 : P];
  __shared__ cplx<R> pxy[SCH ? 3 * P : 1], dzs[SCH ? N : 1], azs[SCH ? N : 1];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const int ntiles = (g.n1 / 2) / TX;
  int u, c;
  unit_comp(ntiles * g.n2, 6, u, c);
  const int tile = u % ntiles, ky = u / ntiles;
  const int kx0 = tile * TX;
  const long long stride_n = (long long)g.n1h * g.n2;
  const long long base = (long long)ky * g.n1h;
  R ty = R(0);
  if constexpr (SCH == 0) z_freqs<R, N, P, NT>(g, kx0, tile, TX, ky, txs, tzs, ty);
  else z_rot<R, N, P, NT>(g, kx0, tile, TX, ky, pxy, dzs, azs);
  // component c = (a, b): xx, yy, zz, yz, xz, xy
  const int ca = (c < 3) ? c : (c == 3 ? 1 : 0);
  const int cb = (c < 3) ? c : (c == 5 ? 1 : 2);
  auto col = [&](int x) -> int {
    if (x < TX) return kx0 + x;
    return (tile == 0) ? g.n1 / 2 : -1;
  };
  auto upd = [&](cplx<R> zz, cplx<R> pp) -> cplx<R> {
    return cplx<R>{(R)((double)zz.x + be * (double)pp.x), (R)((double)zz.y + be * (double)pp.y)};
  };
  __syncthreads();
  for (int t = threadIdx.x; t < P * Nb; t += NT) {
    const int x = t % P, n1 = t / P;
    const int cx = col(x);
    cplx<R> v[Na];
    if (cx >= 0) {
      const R tx = SCH == 0 ? txs[x] : R(0);
      const long long i0 = base + (long long)n1 * stride_n + cx;
      const long long sm = (long long)Nb * stride_n;
      cplx<R> za[Na], pa[Na];
#pragma unroll
      for (int m = 0; m < Na; ++m) {
        za[m] = zv[ca * cs + i0 + m * sm];
        pa[m] = pold[ca * cs + i0 + m * sm];
      }
#pragma unroll
      for (int m = 0; m < Na; ++m) v[m] = upd(za[m], pa[m]);     // p_new_a
      if (c < 3) {
#pragma unroll
        for (int m = 0; m < Na; ++m) {
          pnew[ca * cs + i0 + m * sm] = v[m];
          if constexpr (SCH == 0) {
            const R ta = (ca == 0) ? tx : (ca == 1 ? ty : tzs[n1 + Nb * m]);
            v[m] = imul(ta, v[m]);
          } else {
            const int kz = n1 + Nb * m;
            v[m] = cmul(cmul(pxy[ca * P + x], ca == 2 ? dzs[kz] : azs[kz]), v[m]);
          }
        }
      } else {
        cplx<R> zb[Na], pb[Na];
#pragma unroll
        for (int m = 0; m < Na; ++m) {
          zb[m] = zv[cb * cs + i0 + m * sm];
          pb[m] = pold[cb * cs + i0 + m * sm];
        }
#pragma unroll
        for (int m = 0; m < Na; ++m) {
          const cplx<R> nb = upd(zb[m], pb[m]);
          if constexpr (SCH == 0) {
            const R tz = tzs[n1 + Nb * m];
            const R ta = (ca == 0) ? tx : ty;                // off the diagonal a < b, a < 2
            const R tb = (cb == 1) ? ty : tz;
            v[m] = cscale(cadd(imul(ta, nb), imul(tb, v[m])), R(0.5));
          } else {
            const int kz = n1 + Nb * m;
            const cplx<R> ka = cmul(pxy[ca * P + x], azs[kz]);          // a is x or y
            const cplx<R> kb = cmul(pxy[cb * P + x], cb == 2 ? dzs[kz] : azs[kz]);
            v[m] = cscale(cadd(cmul(ka, nb), cmul(kb, v[m])), R(0.5));
          }
        }
      }
    } else {
#pragma unroll
      for (int m = 0; m < Na; ++m) v[m] = cplx<R>{0, 0};
    }
    reg_dft<R, Na, true>(v);
#pragma unroll
    for (int k2 = 0; k2 < Na; ++k2) {
      cplx<R> w = tw[n1 * k2];
      w.y = -w.y;
      A[x * PITCH + n1 + Nb * k2] = (k2 == 0) ? v[k2] : cmul(v[k2], w);
    }
  }
  __syncthreads();
  cplx<R>* d = e + (long long)c * cs + base;
  for (int t = threadIdx.x; t < P * Na; t += NT) {
    const int x = t % P, k2 = t / P;
    const int cx = col(x);
    cplx<R> v[Nb];
#pragma unroll
    for (int n1 = 0; n1 < Nb; ++n1) v[n1] = A[x * PITCH + n1 + Nb * k2];
    reg_dft<R, Nb, true>(v);
    if (cx >= 0) {
#pragma unroll
      for (int k1 = 0; k1 < Nb; ++k1) d[(long long)(k2 + Na * k1) * stride_n + cx] = v[k1];
    }
  }
}

// Component i of q = -i xi~ . F_z{s} and the block partial of the Parseval-weighted
// <p, q>, in two rounds: xi~_z F_z{s_iz} and F_z{xi~_x s_ix + xi~_y s_iy} (whose x and y
// factors are constant along z); the first round's result waits in LDS.  Components x and
// y take the z round first, component z the other: the three blocks of a work unit (one
// XCD, dispatched together) then read each shared stress component (xz, yz, xy) in the
// same round, so that the second read comes from L2.
template <typename R, int N, int TX, int NT, int SCH>
__global__ void __launch_bounds__(NT)
k_zdiv_fwd(const cplx<R>* __restrict__ s, cplx<R>* __restrict__ q, const cplx<R>* __restrict__ pv,
           long long cs, Grid g, const cplx<R>* __restrict__ tw_g, double* __restrict__ partial,
           const double* __restrict__ stop) {
  {
    const long long d = slot_delta(g);
    s = at_slot(s, d); q = at_slot(q, d); pv = at_slot(pv, d); tw_g = at_slot(tw_g, d);
    partial = at_slot(partial, d); stop = at_slot(stop, d);
  }
  if (stop && *stop != 0.0) return;
  constexpr int P = TX + 1;
  constexpr int Na = ZSplit<N>::Na, Nb = ZSplit<N>::Nb;
  constexpr int PITCH = N + 1;
  __shared__ cplx<R> A[P * PITCH];
  __shared__ cplx<R> D[P * N];
  __shared__ cplx<R> tw[N];
  __shared__ R tzs[SCH ? 1 : N], txs[SCH ? 1 : P];
  __shared__ cplx<R> pxy[SCH ? 3 * P : 1], dzs[SCH ? N : 1], azs[SCH ? N : 1];
  __shared__ double red[NT / 64];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const int ntiles = (g.n1 / 2) / TX;
  int u, i;
  unit_comp(ntiles * g.n2, 3, u, i);
  const int tile = u % ntiles, ky = u / ntiles;
  const int kx0 = tile * TX;
  const long long stride_n = (long long)g.n1h * g.n2;
  const long long base = (long long)ky * g.n1h;
  R ty = R(0);
  if constexpr (SCH == 0) z_freqs<R, N, P, NT>(g, kx0, tile, TX, ky, txs, tzs, ty);
  else z_rot<R, N, P, NT>(g, kx0, tile, TX, ky, pxy, dzs, azs);
  // s_ix, s_iy, s_iz among xx, yy, zz, yz, xz, xy
  const int sx = (i == 0) ? 0 : (i == 1 ? 5 : 4);
  const int sy = (i == 0) ? 5 : (i == 1 ? 1 : 3);
  const int sz = (i == 0) ? 4 : (i == 1 ? 3 : 2);
  auto col = [&](int x) -> int {
    if (x < TX) return kx0 + x;
    return (tile == 0) ? g.n1 / 2 : -1;
  };
  double acc = 0.0;
  __syncthreads();
#pragma unroll
  for (int round = 0; round < 2; ++round) {
    const bool zr = (i == 2) ? (round == 1) : (round == 0);     // the xi~_z round
    for (int t = threadIdx.x; t < P * Nb; t += NT) {
      const int x = t % P, n1 = t / P;
      const int cx = col(x);
      cplx<R> v[Na];
      if (cx >= 0) {
        const long long i0 = base + (long long)n1 * stride_n + cx;
        const long long sm = (long long)Nb * stride_n;
        if (zr) {
#pragma unroll
          for (int m = 0; m < Na; ++m) v[m] = s[sz * cs + i0 + m * sm];
        } else {
          cplx<R> a[Na], b[Na];
#pragma unroll
          for (int m = 0; m < Na; ++m) {
            a[m] = s[sx * cs + i0 + m * sm];
            b[m] = s[sy * cs + i0 + m * sm];
          }
          if constexpr (SCH == 0) {
            const R tx = txs[x];
#pragma unroll
            for (int m = 0; m < Na; ++m) v[m] = cadd(cscale(a[m], tx), cscale(b[m], ty));
          } else {      // conj(Dx Ay) s_ix + conj(Ax Dy) s_iy; conj(Az) follows the DFT
            const cplx<R> fx = pxy[0 * P + x], fy = pxy[1 * P + x];
            const cplx<R> cfx{fx.x, -fx.y}, cfy{fy.x, -fy.y};
#pragma unroll
            for (int m = 0; m < Na; ++m) v[m] = cadd(cmul(cfx, a[m]), cmul(cfy, b[m]));
          }
        }
      } else {
#pragma unroll
        for (int m = 0; m < Na; ++m) v[m] = cplx<R>{0, 0};
      }
      reg_dft<R, Na, false>(v);
#pragma unroll
      for (int k2 = 0; k2 < Na; ++k2)
        A[x * PITCH + n1 + Nb * k2] = (k2 == 0) ? v[k2] : cmul(v[k2], tw[n1 * k2]);
    }
    __syncthreads();
    for (int t = threadIdx.x; t < P * Na; t += NT) {
      const int x = t % P, k2 = t / P;
      const int cx = col(x);
      cplx<R> v[Nb];
#pragma unroll
      for (int n1 = 0; n1 < Nb; ++n1) v[n1] = A[x * PITCH + n1 + Nb * k2];
      reg_dft<R, Nb, false>(v);
      if (cx < 0) continue;
      if constexpr (SCH == 0) {
        if (zr) {
#pragma unroll
          for (int k1 = 0; k1 < Nb; ++k1) v[k1] = cscale(v[k1], tzs[k2 + Na * k1]);
        }
      } else {
        // z round: conj(Ax Ay) conj(Dz) F_z{s_iz}; x-y round: conj(Az) F_z{...}
        const cplx<R> fz = pxy[2 * P + x];
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) {
          const int kz = k2 + Na * k1;
          const cplx<R> f = zr ? cmul(fz, dzs[kz]) : azs[kz];
          v[k1] = cmul(cplx<R>{f.x, -f.y}, v[k1]);
        }
      }
      if (round == 0) {
        // D is private to the thread that owns item (x, k2) in both rounds
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) D[x * N + k2 + Na * k1] = v[k1];
      } else {
        const long long i0 = (long long)i * cs + base + (long long)k2 * stride_n + cx;
        const long long sk = (long long)Na * stride_n;
        cplx<R> pp[Nb];
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) pp[k1] = pv[i0 + k1 * sk];
        double dot = 0.0;
#pragma unroll
        for (int k1 = 0; k1 < Nb; ++k1) {
          const cplx<R> dd = cadd(v[k1], D[x * N + k2 + Na * k1]);
          // spectral: q = -i d; rotated: the conj(k) factors are already applied
          const cplx<R> qq = SCH == 0 ? cplx<R>{dd.y, -dd.x} : dd;
          q[i0 + k1 * sk] = qq;
          dot += (double)pp[k1].x * (double)qq.x + (double)pp[k1].y * (double)qq.y;
        }
        acc += parseval_w(cx, g.n1) * dot;
      }
    }
    __syncthreads();
  }
  block_partial_sum(acc, partial, red);
}

// LDS bytes of the fused z kernels (the rotated scheme adds its factor tables, 3 P + 2 N
// complex)
template <typename R>
constexpr size_t zgrad_lds(int N, int P, int sch) {
  return ((size_t)P * (N + 1) + N) * sizeof(cplx<R>) + (size_t)(N + P) * sizeof(R) +
         (sch ? (size_t)(3 * P + 2 * N) * sizeof(cplx<R>) : 0) + 32 * sizeof(double);
}
template <typename R>
constexpr size_t zdiv_lds(int N, int P, int sch) {
  return ((size_t)P * (N + 1) + (size_t)P * N + N) * sizeof(cplx<R>) +
         (size_t)(N + P) * sizeof(R) + (sch ? (size_t)(3 * P + 2 * N) * sizeof(cplx<R>) : 0) +
         16 * sizeof(double);
}

// LDS ceiling of one fused z block: the whole 160 KB of a gfx950 CU (the 256-point
// columns take one block per CU; the shorter columns stay within kRegLdsMax by their caps)
constexpr size_t kZLdsMax = 160 * 1024;

// Widest x tile (64, 32, 16 or 8 bins plus the Nyquist column) allowed for a column length
// and precision.  Up to 128-point columns: the widest tile that fits for the gradient pass
// (32 bins measured faster than 16; in FP32 64-bin tiles, whose row segments are as long in
// bytes as the FP64 pass's 32-bin ones: 31.1 against 32.4 us at 128^3); the divergence pass
// holds two LDS arrays and runs more blocks per CU at 8 bins (128^3: 47 against 60 us FP64
// at 16 bins, 26 against 34 us FP32 at 32).  256-point columns are bound by the locality
// of their accesses, not by occupancy: the z planes of a 256^2 half spectrum lie 528 KB
// apart (FP64), and a block moves one short row segment per plane and operand across all
// 256 planes (the address translations hit; the requests wait on their data).  Longer
// segments help: one block per CU with 32-bin tiles (FP64 gradient pass) takes 781 against
// 1135 us, 16-bin divergence tiles 608 against 669 us; in FP32 64- and 32-bin tiles 476
// against 633 and 345 against 390 us (a second resident block, at 16 bins with fewer
// registers, gained 1 %).  At 128 points the same widening is slower.
template <typename R>
constexpr int z_tile_cap(int N, bool div) {
  if (N == 256) return div ? (sizeof(R) == 4 ? 32 : 16) : (sizeof(R) == 4 ? 64 : 32);
  return div ? 8 : (sizeof(R) == 4 ? 64 : 32);
}
template <typename R>
constexpr size_t z_lds_max(int N) { return N == 256 ? kZLdsMax : kRegLdsMax; }

// Largest x tile within the cap whose LDS fits; 0 if the grid has no fused z pass (odd
// n1, or n3 without a register DFT).
template <typename R, int N>
static int fused_tile(const Grid& g, bool div) {
  if (g.n1 % 2 != 0 || g.n3 != N) return 0;
  const int half = g.n1 / 2;
  const int cap = z_tile_cap<R>(N, div);
  for (int TX : {64, 32, 16, 8}) {
    if (TX > cap) continue;
    const size_t lds = div ? zdiv_lds<R>(N, TX + 1, g.sch) : zgrad_lds<R>(N, TX + 1, g.sch);
    if (half % TX == 0 && lds <= z_lds_max<R>(N)) return TX;
  }
  return 0;
}

template <int NT_ITEMS>
constexpr int threads_for() {
  return ((NT_ITEMS + 63) / 64) * 64 > 1024 ? 1024 : ((NT_ITEMS + 63) / 64) * 64;
}

template <typename R>
bool fused_z_available(const Plans& p) {
  bool ok = false;
  with_length(p.g.n3, [&]<int NC>() {
    if constexpr (NC > 0) ok = fused_tile<R, NC>(p.g, false) > 0 && fused_tile<R, NC>(p.g, true) > 0;
  });
  return ok;
}

template <typename R>
void launch_zgrad_inv(const Plans& p, const cplx<R>* z, const cplx<R>* pold, cplx<R>* pnew,
                      long long cs, double* sc, int ia, int ib, cplx<R>* e, hipStream_t st,
                      const double* stop, CgCheck ck) {
  const Grid& g = p.g;
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(2, sizeof(R) == 8);
  with_length(g.n3, [&]<int NC>() {
    if constexpr (NC > 0) {
      const int TX = fused_tile<R, NC>(g, false);
      auto go = [&]<int T, int S>() {
        if constexpr (T <= z_tile_cap<R>(NC, false) &&
                      zgrad_lds<R>(NC, T + 1, S) <= z_lds_max<R>(NC)) {
          constexpr int NT = threads_for<(T + 1) * ZSplit<NC>::Nb>();
          const int nblk = (g.n1 / 2 / T) * g.n2 * 6;
          hipLaunchKernelGGL((k_zgrad_inv<R, NC, T, NT, S>), dim3(nblk, 1, p.nslot), dim3(NT), 0, st, z, pold,
                             pnew, cs, sc, ia, ib, e, g, tw, stop, ck);
        }
      };
      auto go2 = [&]<int T>() {
        if (g.sch) go.template operator()<T, 1>();
        else go.template operator()<T, 0>();
      };
      if (TX == 64) go2.template operator()<64>();
      else if (TX == 32) go2.template operator()<32>();
      else if (TX == 16) go2.template operator()<16>();
      else if (TX == 8) go2.template operator()<8>();
    }
  });
}

template <typename R>
int launch_zdiv_fwd(const Plans& p, const cplx<R>* s, cplx<R>* q, const cplx<R>* pv, long long cs,
                    double* partial, hipStream_t st, const double* stop) {
  const Grid& g = p.g;
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(2, sizeof(R) == 8);
  int nblk = 0;
  with_length(g.n3, [&]<int NC>() {
    if constexpr (NC > 0) {
      const int TX = fused_tile<R, NC>(g, true);
      auto go = [&]<int T, int S>() {
        if constexpr (T <= z_tile_cap<R>(NC, true) &&
                      zdiv_lds<R>(NC, T + 1, S) <= z_lds_max<R>(NC)) {
          constexpr int NT = threads_for<(T + 1) * ZSplit<NC>::Nb>();
          nblk = (g.n1 / 2 / T) * g.n2 * 3;
          hipLaunchKernelGGL((k_zdiv_fwd<R, NC, T, NT, S>), dim3(nblk, 1, p.nslot), dim3(NT), 0, st, s, q, pv,
                             cs, g, tw, partial, stop);
        }
      };
      auto go2 = [&]<int T>() {
        if (g.sch) go.template operator()<T, 1>();
        else go.template operator()<T, 0>();
      };
      if (TX == 32) go2.template operator()<32>();
      else if (TX == 16) go2.template operator()<16>();
      else if (TX == 8) go2.template operator()<8>();
    }
  });
  return nblk;
}

hipError_t upload_reg_twiddles_zfused(hipStream_t st) { return fill_reg_twiddles(st); }

#define RVE_ZFUSED_INST(R)                                                                       \
  template bool fused_z_available<R>(const Plans&);                                              \
  template void launch_zgrad_inv<R>(const Plans&, const cplx<R>*, const cplx<R>*, cplx<R>*,       \
                                    long long, double*, int, int, cplx<R>*, hipStream_t,         \
                                    const double*, CgCheck);                                     \
  template int launch_zdiv_fwd<R>(const Plans&, const cplx<R>*, cplx<R>*, const cplx<R>*,         \
                                  long long, double*, hipStream_t, const double*);

RVE_ZFUSED_INST(double)
RVE_ZFUSED_INST(float)

}  // namespace rvefft
