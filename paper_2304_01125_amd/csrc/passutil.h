// Helpers shared by the pass translation units: Hermitian row access and row
// bookkeeping of the x passes (device), LDS budgets and the compile-time length
// dispatch of the launchers (host).
#pragma once
#include "kernels.h"
#include "fft.h"
#include "regfft.h"

namespace rvefft {

template <typename R>
__device__ __forceinline__ void load_twiddles(cplx<R>* tw_s, const cplx<R>* tw_g, int n) {
  for (int t = threadIdx.x; t < n; t += blockDim.x) tw_s[t] = tw_g[t];
}

// Half-spectrum bin k of a real row, read as a Hermitian row (imaginary parts of bin
// 0 and of the Nyquist bin dropped: they do not exist for a real row).
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

template <typename R, int NC>
__device__ __forceinline__ cplx<R>* row_fft(cplx<R>* A, cplx<R>* B, const cplx<R>* tw,
                                            const AxisPlan& pl, int P, bool inv) {
  if constexpr (NC > 0) return fft_rows_ct<R, NC>(A, B, tw, P, inv);
  else return fft_pencils<R, false>(A, B, tw, pl, P, 1, pl.n + 1, inv);
}

constexpr int kMaxRowPairs = 32;

// Per-pencil row bookkeeping of the x passes: pencil p of the block packs the rows
// r0 = 2(pair0+p) and r1 = r0+1 of the flattened (component, k, j) order.
struct RowPair {
  long long c0, rem0, c1, rem1;   // component and voxel row of each real row (-1: none)
};

__device__ __forceinline__ void row_pairs(RowPair* rp, int P, long long pair0, long long rows_per_comp,
                                          long long nrows) {
  for (int p = threadIdx.x; p < P; p += blockDim.x) {
    const long long r0 = 2 * (pair0 + p), r1 = r0 + 1;
    RowPair q;
    q.c0 = (r0 < nrows) ? r0 / rows_per_comp : -1;
    q.rem0 = (r0 < nrows) ? r0 % rows_per_comp : 0;
    q.c1 = (r1 < nrows) ? r1 / rows_per_comp : -1;
    q.rem1 = (r1 < nrows) ? r1 % rows_per_comp : 0;
    rp[p] = q;
  }
}

// ---------------------------------------------------------------------------
// Host launch helpers.
constexpr size_t kLdsBudget = 64 * 1024;

inline size_t xpass_smem(int n1, int P, size_t csz) {
  return ((size_t)n1 + (size_t)P * (n1 + 1) * 2) * csz;
}

template <typename R>
inline int pick_rows(int n1, int maxP) {
  int P = maxP;
  while (P > 1 && xpass_smem(n1, P, sizeof(cplx<R>)) > kLdsBudget) P /= 2;
  return P;
}

// Calls F.template operator()<NC>() with the compile-time length of n (0 if none).
template <typename F>
inline void with_length(int n, F&& f) {
  switch (n) {
    case 16: f.template operator()<16>(); break;
    case 32: f.template operator()<32>(); break;
    case 48: f.template operator()<48>(); break;
    case 64: f.template operator()<64>(); break;
    case 96: f.template operator()<96>(); break;
    case 128: f.template operator()<128>(); break;
    case 256: f.template operator()<256>(); break;
    default: f.template operator()<0>(); break;
  }
}

// LDS ceiling of the register-DFT pass kernels (static LDS per block)
constexpr size_t kRegLdsMax = 80 * 1024;

}  // namespace rvefft
