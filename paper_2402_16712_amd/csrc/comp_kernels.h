// comp_kernels.h -- successive components (Sec. 2, after Algorithm 3): each
// component is Algorithm 1 on the data projected onto the null space of the
// components found before it.  The kernels here do the projection:
//   w_c = v_c made orthogonal to w_0 .. w_{c-1} (classical Gram-Schmidt,
//         unnormalised): w_k = fl(w_k - fl(fl(R64(w_l . v_c) / |w_l|^2) * w_lk))
//   y_ik = fl(y_ik - fl(s_i * u_k)),  s_i = R64_k fl(y_ik * w_ck),
//         u_k = fl(w_ck / |w_c|^2),  |w|^2 = R64_k fl(w_k * w_k)
// Every product is rounded on its own (no fused multiply-add) and every dot
// product uses the R64 order, so the result is defined bit for bit.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fit_kernels.h"

// Y (n x m, ld n) = X (n x m, ld ld)
__global__ void k_copy_matrix(const double *__restrict__ X, long long ld, int n, int m, double *__restrict__ Y) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * m) return;
  const int k = (int)(e / n), i = (int)(e % n);
  Y[e] = X[(long long)k * ld + i];
}

// R64 dot product of two m-vectors by one wave (result on every lane)
__device__ __forceinline__ double wave_r64_dot(const double *a, const double *b, int m, int lane) {
  double p = 0.0;
  for (int k = lane; k < m; k += 64) {
    const double t = a[k] * b[k];
    p = p + t;
  }
  return __shfl(wave_r64_tree(p), 0);
}

// Gram-Schmidt of component c (one wave): W[c*m..] = w_c, cw[c] = |w_c|^2,
// U = w_c / |w_c|^2; flag = 1 when w_c = 0 (v_c lies in the span of the
// earlier components)
__global__ void __launch_bounds__(64) k_gs(const double *__restrict__ v, double *__restrict__ W,
                                           double *__restrict__ cw, int c, int m, double *__restrict__ U,
                                           int *__restrict__ flag) {
  const int lane = threadIdx.x;
  double *w = W + (long long)c * m;
  for (int k = lane; k < m; k += 64) w[k] = v[k];
  __syncthreads();
  for (int l = 0; l < c; ++l) {
    const double *wl = W + (long long)l * m;
    const double coef = wave_r64_dot(wl, v, m, lane) / cw[l];
    for (int k = lane; k < m; k += 64) {
      const double prod = coef * wl[k];
      w[k] = w[k] - prod;
    }
    __syncthreads();
  }
  const double nn = wave_r64_dot(w, w, m, lane);
  if (lane == 0) {
    cw[c] = nn;
    *flag = (nn > 0.0) ? 0 : 1;
  }
  for (int k = lane; k < m; k += 64) U[k] = w[k] / nn;
}

// s_i = R64_k fl(y_ik w_k), one wave per row
__global__ void __launch_bounds__(256) k_rowdot(const double *__restrict__ Y, int n, int m,
                                                const double *__restrict__ w, double *__restrict__ s) {
  const int i = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (i >= n) return;
  double p = 0.0;
  for (int k = lane; k < m; k += 64) {
    const double t = Y[(long long)k * n + i] * w[k];
    p = p + t;
  }
  const double r = wave_r64_tree(p);
  if (lane == 0) s[i] = r;
}

// y_ik = fl(y_ik - fl(s_i u_k))
__global__ void k_deflate(double *__restrict__ Y, int n, int m, const double *__restrict__ s,
                          const double *__restrict__ U) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * m) return;
  const int k = (int)(e / n), i = (int)(e % n);
  const double prod = s[i] * U[k];
  Y[e] = Y[e] - prod;
}

// status of the whole call, as the components are visited in order: the
// first fit error other than ERANGE stops, ERANGE is remembered, a zero
// projection (flag) stops with EINVAL
__global__ void k_comp_status(const int *__restrict__ cstat, const int *__restrict__ gsflag, int p,
                              int *__restrict__ status, int *__restrict__ sticky) {
  if (threadIdx.x != 0) return;
  int st = L1LINE_OK;
  for (int c = 0; c < p; ++c) {
    const int f = cstat[c];
    if (f != L1LINE_OK && f != L1LINE_ERANGE) {
      st = f;
      break;
    }
    if (f == L1LINE_ERANGE) st = f;
    if (c < p - 1 && gsflag[c]) {
      st = L1LINE_EINVAL;
      break;
    }
  }
  if (status) *status = st;
  if (sticky && st != L1LINE_OK) atomicCAS(sticky, 0, st);
}
