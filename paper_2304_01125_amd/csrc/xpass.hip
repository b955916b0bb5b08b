// x passes of the 3-D real transforms (Sec. 3.1): real rows <-> half-spectrum rows,
// two real rows packed per complex pencil.  The fused tangent pass applies the degraded
// tangent g K : eps between the inverse and the forward row transforms, the real-space
// factor of the linearised equilibrium operator (eq. newton).
#include "passutil.h"
#include <hip/hip_ext.h>

namespace rvefft {

// ---------------------------------------------------------------------------
// x pass, real -> half spectrum (optionally multiplying the input by g(phi)).
template <typename R, typename TI, int NC>
__global__ void __launch_bounds__(256)
k_x_r2c(const TI* __restrict__ in, long long in_cs, const double* __restrict__ phi, double kres,
        cplx<R>* __restrict__ out, long long out_cs, int ncomp, Grid g, AxisPlan pl,
        const cplx<R>* __restrict__ tw_g, int P, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  __shared__ RowPair rp[kMaxRowPairs];
  const int N = NC > 0 ? NC : g.n1;
  const int NH = N / 2 + 1, pitch = N + 1;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long rows_per_comp = (long long)g.n2 * g.n3;
  row_pairs(rp, P, (long long)blockIdx.x * P, rows_per_comp, rows_per_comp * ncomp);
  __syncthreads();
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, i = t % N;
    const RowPair q = rp[p];
    R a = 0, b = 0;
    if (q.c0 >= 0) {
      const long long v = q.rem0 * N + i;
      double x = (double)in[q.c0 * in_cs + v];
      if (phi) { const double u = 1.0 - phi[v]; x *= u * u + kres; }
      a = (R)x;
    }
    if (q.c1 >= 0) {
      const long long v = q.rem1 * N + i;
      double x = (double)in[q.c1 * in_cs + v];
      if (phi) { const double u = 1.0 - phi[v]; x *= u * u + kres; }
      b = (R)x;
    }
    A[p * pitch + i] = cplx<R>{a, b};
  }
  __syncthreads();
  cplx<R>* Z = row_fft<R, NC>(A, B, tw, pl, P, false);
  for (int t = threadIdx.x; t < P * NH; t += blockDim.x) {
    const int p = t / NH, k = t % NH;
    const RowPair q = rp[p];
    if (q.c0 < 0) continue;
    const cplx<R> zk = Z[p * pitch + k];
    const cplx<R> zm = Z[p * pitch + ((N - k) % N)];
    // A_k = (Z_k + conj Z_-k)/2 ; B_k = (Z_k - conj Z_-k)/(2i)
    out[q.c0 * out_cs + q.rem0 * NH + k] = cplx<R>{R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    if (q.c1 >= 0)
      out[q.c1 * out_cs + q.rem1 * NH + k] =
          cplx<R>{R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
  }
}

// x pass, half spectrum -> real: out = scale * x (or out += scale * x).
template <typename R, typename TO, int NC>
__global__ void __launch_bounds__(256)
k_x_c2r(const cplx<R>* __restrict__ in, long long in_cs, TO* __restrict__ out, long long out_cs,
        int ncomp, double scale, int accumulate, Grid g, AxisPlan pl,
        const cplx<R>* __restrict__ tw_g, int P, const double* __restrict__ stop) {
  if (stop && *stop != 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  __shared__ RowPair rp[kMaxRowPairs];
  const int N = NC > 0 ? NC : g.n1;
  const int NH = N / 2 + 1, pitch = N + 1;
  cplx<R>* tw = reinterpret_cast<cplx<R>*>(smem_raw);
  cplx<R>* A = tw + N;
  cplx<R>* B = A + P * pitch;
  load_twiddles(tw, tw_g, N);
  const long long rows_per_comp = (long long)g.n2 * g.n3;
  row_pairs(rp, P, (long long)blockIdx.x * P, rows_per_comp, rows_per_comp * ncomp);
  __syncthreads();
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, k = t % N;
    const RowPair q = rp[p];
    cplx<R> a = {0, 0}, b = {0, 0};
    if (q.c0 >= 0) a = herm_bin(in + q.c0 * in_cs + q.rem0 * NH, k, N);
    if (q.c1 >= 0) b = herm_bin(in + q.c1 * in_cs + q.rem1 * NH, k, N);
    A[p * pitch + k] = cplx<R>{a.x - b.y, a.y + b.x};     // a + i b
  }
  __syncthreads();
  cplx<R>* Z = row_fft<R, NC>(A, B, tw, pl, P, true);
  for (int t = threadIdx.x; t < P * N; t += blockDim.x) {
    const int p = t / N, i = t % N;
    const RowPair q = rp[p];
    if (q.c0 < 0) continue;
    const cplx<R> z = Z[p * pitch + i];
    {
      TO* o = out + q.c0 * out_cs + q.rem0 * N + i;
      const double v = scale * (double)z.x;
      *o = accumulate ? (TO)((double)*o + v) : (TO)v;
    }
    if (q.c1 >= 0) {
      TO* o = out + q.c1 * out_cs + q.rem1 * N + i;
      const double v = scale * (double)z.y;
      *o = accumulate ? (TO)((double)*o + v) : (TO)v;
    }
  }
}

// Fused x pass of the equilibrium operator on 6 components (in place):
//   eps = F_x^-1{.}, sigma = scale * gK : eps (Mandel), out = F_x{sigma}.
// One block holds Q voxel rows; components (xx,yy), (zz,yz), (xz,xy) share pencils.
template <typename R, int NC>
__global__ void __launch_bounds__(256)
k_x_tangent(cplx<R>* __restrict__ data, long long cs, const R* __restrict__ gK, double scale,
            Grid g, AxisPlan pl, const cplx<R>* __restrict__ tw_g, int Q,
            const double* __restrict__ stop) {
  {
    const long long d = slot_delta(g);
    data = at_slot(data, d); gK = at_slot(gK, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
  }
  if (stop && *stop != 0.0) return;
  extern __shared__ unsigned char smem_raw[];
  const int N = NC > 0 ? NC : g.n1;
  const int NH = N / 2 + 1, pitch = N + 1;
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
  cplx<R>* Z = row_fft<R, NC>(A, B, tw, pl, P, true);
  cplx<R>* W = (Z == A) ? B : A;
  const R s2 = (R)1.41421356237309504880;
  const R is2 = (R)0.70710678118654752440;
  for (int t = threadIdx.x; t < Q * N; t += blockDim.x) {
    const int q = t / N, i = t % N;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const long long v = rem * N + i;
    const cplx<R> z0 = Z[(3 * q + 0) * pitch + i];
    const cplx<R> z1 = Z[(3 * q + 1) * pitch + i];
    const cplx<R> z2 = Z[(3 * q + 2) * pitch + i];
    const R e[6] = {z0.x, z0.y, z1.x, s2 * z1.y, s2 * z2.x, s2 * z2.y};   // Mandel strain
    R s[6] = {0, 0, 0, 0, 0, 0};
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) {
        const R k = gK[(long long)idx * g.nvox + v];
        s[a] += k * e[b];
        if (b != a) s[b] += k * e[a];
        ++idx;
      }
    const R sc = (R)scale;
    W[(3 * q + 0) * pitch + i] = cplx<R>{sc * s[0], sc * s[1]};
    W[(3 * q + 1) * pitch + i] = cplx<R>{sc * s[2], sc * is2 * s[3]};
    W[(3 * q + 2) * pitch + i] = cplx<R>{sc * is2 * s[4], sc * is2 * s[5]};
  }
  __syncthreads();
  cplx<R>* other = (W == A) ? B : A;
  cplx<R>* Y = row_fft<R, NC>(W, other, tw, pl, P, false);
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

// Fused tangent x pass with a compile-time row length and rows per block, single LDS
// buffer (in-place Stockham stages, fft.h): same arithmetic as k_x_tangent.
template <typename R, int N, int Q, int NT>
__global__ void __launch_bounds__(NT)
k_x_tangent_ip(cplx<R>* __restrict__ data, long long cs, const R* __restrict__ gK, double scale,
               Grid g, const cplx<R>* __restrict__ tw_g, const double* __restrict__ stop) {
  {
    const long long d = slot_delta(g);
    data = at_slot(data, d); gK = at_slot(gK, d); tw_g = at_slot(tw_g, d); stop = at_slot(stop, d);
  }
  if (stop && *stop != 0.0) return;
  constexpr int NH = N / 2 + 1, PITCH = N + 1, P = 3 * Q;
  __shared__ cplx<R> tw[N];
  __shared__ cplx<R> A[P * PITCH];
  for (int t = threadIdx.x; t < N; t += NT) tw[t] = tw_g[t];
  const long long nrows = (long long)g.n2 * g.n3;
  // blocks go to the 8 XCDs in turn: when the count allows, XCD j takes a contiguous range
  // of rows, so that neighbouring rows (rows of N/2 + 1 bins share the 128-B line at their
  // boundary) meet in its L2
  long long bid = blockIdx.x;
  if ((gridDim.x & 7) == 0) bid = (bid & 7) * (gridDim.x >> 3) + (bid >> 3);
  const long long row0 = bid * Q;
  for (int t = threadIdx.x; t < P * N; t += NT) {
    const int p = t / N, k = t % N;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    cplx<R> a = {0, 0}, b = {0, 0};
    if (rem < nrows) {
      a = herm_bin(data + (2 * pair) * cs + rem * NH, k, N);
      b = herm_bin(data + (2 * pair + 1) * cs + rem * NH, k, N);
    }
    A[p * PITCH + k] = cplx<R>{a.x - b.y, a.y + b.x};
  }
  __syncthreads();
  ct_run_ip<R, N, 0, 1, 1, PITCH, P, false, NT>(A, tw, true);
  const R s2 = (R)1.41421356237309504880;
  const R is2 = (R)0.70710678118654752440;
  const R sc = (R)scale;
  for (int t = threadIdx.x; t < Q * N; t += NT) {
    const int q = t / N, i = t % N;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const long long v = rem * N + i;
    const cplx<R> z0 = A[(3 * q + 0) * PITCH + i];
    const cplx<R> z1 = A[(3 * q + 1) * PITCH + i];
    const cplx<R> z2 = A[(3 * q + 2) * PITCH + i];
    const R e[6] = {z0.x, z0.y, z1.x, s2 * z1.y, s2 * z2.x, s2 * z2.y};
    R s[6] = {0, 0, 0, 0, 0, 0};
    int idx = 0;
#pragma unroll
    for (int a = 0; a < 6; ++a)
#pragma unroll
      for (int b = a; b < 6; ++b) {
        // the tangent streams through once per pass: non-temporal loads keep it from
        // displacing the spectra that neighbouring rows and the next pass read from L2 and
        // the Infinity Cache (at 128^3: 99 against 116 us FP64, 57 against 62 us FP32)
        const R k = __builtin_nontemporal_load(gK + (long long)idx * g.nvox + v);
        s[a] += k * e[b];
        if (b != a) s[b] += k * e[a];
        ++idx;
      }
    A[(3 * q + 0) * PITCH + i] = cplx<R>{sc * s[0], sc * s[1]};
    A[(3 * q + 1) * PITCH + i] = cplx<R>{sc * s[2], sc * is2 * s[3]};
    A[(3 * q + 2) * PITCH + i] = cplx<R>{sc * is2 * s[4], sc * is2 * s[5]};
  }
  __syncthreads();
  ct_run_ip<R, N, 0, 1, 1, PITCH, P, false, NT>(A, tw, false);
  for (int t = threadIdx.x; t < P * NH; t += NT) {
    const int p = t / NH, k = t % NH;
    const int q = p / 3, pair = p % 3;
    const long long rem = row0 + q;
    if (rem >= nrows) continue;
    const cplx<R> zk = A[p * PITCH + k];
    const cplx<R> zm = A[p * PITCH + ((N - k) % N)];
    data[(2 * pair) * cs + rem * NH + k] = cplx<R>{R(0.5) * (zk.x + zm.x), R(0.5) * (zk.y - zm.y)};
    data[(2 * pair + 1) * cs + rem * NH + k] =
        cplx<R>{R(0.5) * (zk.y + zm.y), R(-0.5) * (zk.x - zm.x)};
  }
}

template <typename R>
void launch_x_r2c(const Plans& p, const void* in, bool in_f64, long long in_cs, const double* phi,
                  double kres, cplx<R>* out, long long out_cs, int ncomp, hipStream_t st,
                  const double* stop) {
  const Grid& g = p.g;
  const int P = pick_rows<R>(g.n1, 16);
  const long long pairs = ((long long)g.n2 * g.n3 * ncomp + 1) / 2;
  const int nblk = (int)((pairs + P - 1) / P);
  const size_t sm = xpass_smem(g.n1, P, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  with_length(g.n1, [&]<int NC>() {
    if (in_f64)
      hipLaunchKernelGGL((k_x_r2c<R, double, NC>), dim3(nblk), dim3(256), sm, st,
                         (const double*)in, in_cs, phi, kres, out, out_cs, ncomp, g, p.ax[0], tw, P, stop);
    else
      hipLaunchKernelGGL((k_x_r2c<R, float, NC>), dim3(nblk), dim3(256), sm, st, (const float*)in,
                         in_cs, phi, kres, out, out_cs, ncomp, g, p.ax[0], tw, P, stop);
  });
}

template <typename R>
void launch_x_c2r(const Plans& p, const cplx<R>* in, long long in_cs, void* out, bool out_f64,
                  long long out_cs, int ncomp, double scale, int accumulate, hipStream_t st,
                  const double* stop) {
  const Grid& g = p.g;
  const int P = pick_rows<R>(g.n1, 16);
  const long long pairs = ((long long)g.n2 * g.n3 * ncomp + 1) / 2;
  const int nblk = (int)((pairs + P - 1) / P);
  const size_t sm = xpass_smem(g.n1, P, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  with_length(g.n1, [&]<int NC>() {
    if (out_f64)
      hipLaunchKernelGGL((k_x_c2r<R, double, NC>), dim3(nblk), dim3(256), sm, st, in, in_cs,
                         (double*)out, out_cs, ncomp, scale, accumulate, g, p.ax[0], tw, P, stop);
    else
      hipLaunchKernelGGL((k_x_c2r<R, float, NC>), dim3(nblk), dim3(256), sm, st, in, in_cs,
                         (float*)out, out_cs, ncomp, scale, accumulate, g, p.ax[0], tw, P, stop);
  });
}

// With ev0/ev1 set, the launch itself timestamps its start and end into them (the
// benchmark's live timing of this pass).
template <typename R>
void launch_x_tangent(const Plans& p, cplx<R>* data, long long cs, const R* gK, double scale,
                      hipStream_t st, const double* stop, hipEvent_t ev0, hipEvent_t ev1) {
  const Grid& g = p.g;
  int Q = 8;
  while (Q > 1 && xpass_smem(g.n1, 3 * Q, sizeof(cplx<R>)) > kLdsBudget) Q /= 2;
  const long long rows = (long long)g.n2 * g.n3;
  const int nblk = (int)((rows + Q - 1) / Q);
  const size_t sm = xpass_smem(g.n1, 3 * Q, sizeof(cplx<R>));
  const cplx<R>* tw = (const cplx<R>*)p.tw_ptr(0, sizeof(R) == 8);
  bool done = false;
  with_length(g.n1, [&]<int NC>() {
    if constexpr (NC > 0) {
      // rows per block and block size, from sweeps at 128^3 (FP64 and FP32)
      auto go = [&]<int QI, int NT>() {
        constexpr size_t lds = ((size_t)NC + 3 * QI * (NC + 1)) * sizeof(cplx<R>);
        if constexpr (lds <= 64 * 1024) {
          const int nb = (int)((rows + QI - 1) / QI);
          if (ev0)
            hipExtLaunchKernelGGL((k_x_tangent_ip<R, NC, QI, NT>), dim3(nb, 1, p.nslot), dim3(NT), 0, st, ev0,
                                  ev1, 0, data, cs, gK, scale, g, tw, stop);
          else
            hipLaunchKernelGGL((k_x_tangent_ip<R, NC, QI, NT>), dim3(nb, 1, p.nslot), dim3(NT), 0, st, data,
                               cs, gK, scale, g, tw, stop);
          done = true;
        }
      };
      if constexpr (NC <= 64) go.template operator()<8, 256>();
      else if constexpr (NC >= 256) go.template operator()<1, 256>();   // 967 against 992 us at 256^3
      else go.template operator()<1, 128>();
    }
  });
  if (done) return;
  if (ev0)
    hipExtLaunchKernelGGL((k_x_tangent<R, 0>), dim3(nblk, 1, p.nslot), dim3(256), sm, st, ev0, ev1, 0, data, cs,
                          gK, scale, g, p.ax[0], tw, Q, stop);
  else
    hipLaunchKernelGGL((k_x_tangent<R, 0>), dim3(nblk, 1, p.nslot), dim3(256), sm, st, data, cs, gK, scale, g,
                       p.ax[0], tw, Q, stop);
}

#define RVE_XPASS_INST(R)                                                                        \
  template void launch_x_r2c<R>(const Plans&, const void*, bool, long long, const double*, double, \
                                cplx<R>*, long long, int, hipStream_t, const double*);           \
  template void launch_x_c2r<R>(const Plans&, const cplx<R>*, long long, void*, bool, long long,  \
                                int, double, int, hipStream_t, const double*);                   \
  template void launch_x_tangent<R>(const Plans&, cplx<R>*, long long, const R*, double,          \
                                    hipStream_t, const double*, hipEvent_t, hipEvent_t);

RVE_XPASS_INST(double)
RVE_XPASS_INST(float)

}  // namespace rvefft
