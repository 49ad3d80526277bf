// ranker_kernels.h -- learned candidate ranker for the exhaustive search over
// the preserved coordinate j: per-column features, a 32 -> 128 -> 128 -> 1 MLP
// (BF16 operands on the MFMA units, FP32 accumulation) with its backward pass
// and Adam, and the top-K candidate selection.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <l1line.h>

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------ parameters
// Flat FP32 parameter vector (master weights):
constexpr int MLP_IN = L1LINE_FEATURES, MLP_H = 128;
constexpr int OFF_W1 = 0;                          // [MLP_IN][MLP_H]
constexpr int OFF_B1 = OFF_W1 + MLP_IN * MLP_H;    // [MLP_H]
constexpr int OFF_W2 = OFF_B1 + MLP_H;             // [MLP_H][MLP_H]
constexpr int OFF_B2 = OFF_W2 + MLP_H * MLP_H;     // [MLP_H]
constexpr int OFF_W3 = OFF_B2 + MLP_H;             // [MLP_H]
constexpr int OFF_B3 = OFF_W3 + MLP_H;             // [1]
constexpr int MLP_NPARAM = OFF_B3 + 1;
static_assert(MLP_NPARAM == L1LINE_MLP_PARAMS, "parameter count");

__device__ __forceinline__ float bf16_round(float x) { return (float)(__bf16)x; }

// MFMA 16x16x32 (BF16 in, FP32 accumulate).  Fragment layouts of one wave64:
//   A (16 x 32): lane l holds A[l & 15][8 (l >> 4) + q], q = 0..7
//   B (32 x 16): lane l holds B[8 (l >> 4) + q][l & 15]
//   C (16 x 16): lane l holds C[4 (l >> 4) + q][l & 15], q = 0..3
// A[r][k] = M[(r0 + r) * rs + (k0 + k) * cs]
__device__ __forceinline__ bf16x8 frag_a(const float *M, int rs, int cs, int r0, int k0, int lane) {
  bf16x8 a;
  const int r = r0 + (lane & 15), kb = k0 + 8 * (lane >> 4);
#pragma unroll
  for (int q = 0; q < 8; ++q) a[q] = (__bf16)M[r * rs + (kb + q) * cs];
  return a;
}
// B[k][c] = N[(k0 + k) * rs + (c0 + c) * cs]
__device__ __forceinline__ bf16x8 frag_b(const float *N, int rs, int cs, int k0, int c0, int lane) {
  bf16x8 b;
  const int c = c0 + (lane & 15), kb = k0 + 8 * (lane >> 4);
#pragma unroll
  for (int q = 0; q < 8; ++q) b[q] = (__bf16)N[(kb + q) * rs + c * cs];
  return b;
}
__device__ __forceinline__ f32x4 mfma16(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// ------------------------------------------------------------------ forward
// One wave per 16-row tile:
//   H1 = bf16(relu(bf16(F) bf16(W1) + b1)),  H2 = bf16(relu(H1 bf16(W2) + b2)),
//   out = sum_c H2[c] bf16(W3[c]) + b3  (four 32-column partials added in order)
// H1, H2 (N x 128, the rounded values) are stored when the pointers are given.
constexpr int FWD_ROWS = 16;

__global__ void __launch_bounds__(64)
k_mlp_fwd(const float *__restrict__ P, const float *__restrict__ F, int N, float *__restrict__ out,
          float *__restrict__ H1g, float *__restrict__ H2g) {
  __shared__ float sF[FWD_ROWS * MLP_IN];
  __shared__ float sH1[FWD_ROWS * MLP_H];
  __shared__ float sH2[FWD_ROWS * MLP_H];
  const int lane = threadIdx.x;
  const int row0 = blockIdx.x * FWD_ROWS;
  for (int e = lane; e < FWD_ROWS * MLP_IN; e += 64) {
    const int r = e / MLP_IN, k = e % MLP_IN;
    sF[e] = (row0 + r < N) ? F[(long long)(row0 + r) * MLP_IN + k] : 0.0f;
  }
  __syncthreads();
  const int col = lane & 15, rq = 4 * (lane >> 4);
  for (int cb = 0; cb < MLP_H / 16; ++cb) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    c = mfma16(frag_a(sF, MLP_IN, 1, 0, 0, lane), frag_b(P + OFF_W1, MLP_H, 1, 0, 16 * cb, lane), c);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float h = c[q] + P[OFF_B1 + 16 * cb + col];
      sH1[(rq + q) * MLP_H + 16 * cb + col] = bf16_round(h > 0.f ? h : 0.f);
    }
  }
  __syncthreads();
  for (int cb = 0; cb < MLP_H / 16; ++cb) {
    f32x4 c = {0.f, 0.f, 0.f, 0.f};
    for (int kc = 0; kc < MLP_H / 32; ++kc)
      c = mfma16(frag_a(sH1, MLP_H, 1, 0, 32 * kc, lane), frag_b(P + OFF_W2, MLP_H, 1, 32 * kc, 16 * cb, lane), c);
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const float h = c[q] + P[OFF_B2 + 16 * cb + col];
      sH2[(rq + q) * MLP_H + 16 * cb + col] = bf16_round(h > 0.f ? h : 0.f);
    }
  }
  __syncthreads();
  // output: lane (r = lane & 15, s = lane >> 4) sums columns [32 s, 32 s + 32)
  const int r = lane & 15, sg = lane >> 4;
  float p = 0.f;
  for (int c2 = 32 * sg; c2 < 32 * sg + 32; ++c2) p += sH2[r * MLP_H + c2] * bf16_round(P[OFF_W3 + c2]);
  const float p1 = __shfl(p, r + 16), p2 = __shfl(p, r + 32), p3 = __shfl(p, r + 48);
  if (lane < 16 && row0 + r < N) out[row0 + r] = (((p + p1) + p2) + p3) + P[OFF_B3];
  if (H1g || H2g) {
    for (int e = lane; e < FWD_ROWS * MLP_H; e += 64) {
      const int rr = e / MLP_H;
      if (row0 + rr < N) {
        if (H1g) H1g[(long long)row0 * MLP_H + e] = sH1[e];
        if (H2g) H2g[(long long)row0 * MLP_H + e] = sH2[e];
      }
    }
  }
}

// ----------------------------------------------------------------- backward
// Loss = mean over rows of (out - y)^2.  One wave per 32-row tile writes its
// gradient partial (all parameters) and loss partial; a second kernel adds
// the partials in tile order (deterministic).  Backward products use BF16
// operands (the rounded activations and BF16(dH)) with FP32 accumulation.
constexpr int BWD_ROWS = 32;

__global__ void __launch_bounds__(64)
k_mlp_bwd(const float *__restrict__ P, const float *__restrict__ F, const float *__restrict__ y, int N,
          const float *__restrict__ out, const float *__restrict__ H1g, const float *__restrict__ H2g,
          float *__restrict__ gpart, float *__restrict__ lpart) {
  extern __shared__ __attribute__((aligned(16))) float smem_f[];
  float *sF = smem_f;                         // 32 x 32
  float *sH1 = sF + BWD_ROWS * MLP_IN;        // 32 x 128
  float *sH2 = sH1 + BWD_ROWS * MLP_H;        // 32 x 128
  float *sD2 = sH2 + BWD_ROWS * MLP_H;        // dH2, BF16-rounded, 32 x 128
  float *sD1 = sD2 + BWD_ROWS * MLP_H;        // dH1, BF16-rounded, 32 x 128
  float *sdo = sD1 + BWD_ROWS * MLP_H;        // dout, 32
  const int lane = threadIdx.x;
  const int tile = blockIdx.x, row0 = tile * BWD_ROWS;
  float *g = gpart + (long long)tile * MLP_NPARAM;
  for (int e = lane; e < BWD_ROWS * MLP_IN; e += 64) {
    const int r = e / MLP_IN;
    sF[e] = (row0 + r < N) ? F[(long long)row0 * MLP_IN + e] : 0.0f;
  }
  for (int e = lane; e < BWD_ROWS * MLP_H; e += 64) {
    const int r = e / MLP_H;
    const bool in = row0 + r < N;
    sH1[e] = in ? H1g[(long long)row0 * MLP_H + e] : 0.0f;
    sH2[e] = in ? H2g[(long long)row0 * MLP_H + e] : 0.0f;
  }
  if (lane < BWD_ROWS) {
    const int r = row0 + lane;
    const float d = r < N ? out[r] - y[r] : 0.0f;
    sdo[lane] = 2.0f * d / (float)N;
  }
  __syncthreads();
  if (lane == 0) {
    float l = 0.f;
    for (int r = 0; r < BWD_ROWS; ++r) {
      const int rr = row0 + r;
      const float d = rr < N ? out[rr] - y[rr] : 0.0f;
      l += d * d;
    }
    lpart[tile] = l / (float)N;
    float db3 = 0.f;
    for (int r = 0; r < BWD_ROWS; ++r) db3 += sdo[r];
    g[OFF_B3] = db3;
  }
  // dW3, dH2
  for (int c = lane; c < MLP_H; c += 64) {
    float acc = 0.f;
    const float w3 = bf16_round(P[OFF_W3 + c]);
    for (int r = 0; r < BWD_ROWS; ++r) {
      acc += sH2[r * MLP_H + c] * sdo[r];
      sD2[r * MLP_H + c] = bf16_round(sH2[r * MLP_H + c] > 0.f ? sdo[r] * w3 : 0.f);
    }
    g[OFF_W3 + c] = acc;
  }
  __syncthreads();
  const int col = lane & 15, rq = 4 * (lane >> 4);
  // dW2[i][o] = sum_r H1[r][i] dH2[r][o]
  for (int ib = 0; ib < MLP_H / 16; ++ib)
    for (int ob = 0; ob < MLP_H / 16; ++ob) {
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      c = mfma16(frag_a(sH1, 1, MLP_H, 16 * ib, 0, lane), frag_b(sD2, MLP_H, 1, 0, 16 * ob, lane), c);
#pragma unroll
      for (int q = 0; q < 4; ++q) g[OFF_W2 + (16 * ib + rq + q) * MLP_H + 16 * ob + col] = c[q];
    }
  // db2
  for (int o = lane; o < MLP_H; o += 64) {
    float acc = 0.f;
    for (int r = 0; r < BWD_ROWS; ++r) acc += sD2[r * MLP_H + o];
    g[OFF_B2 + o] = acc;
  }
  // dH1[r][i] = relu'(H1) sum_o dH2[r][o] W2[i][o]
  for (int rb = 0; rb < BWD_ROWS / 16; ++rb)
    for (int ib = 0; ib < MLP_H / 16; ++ib) {
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      for (int kc = 0; kc < MLP_H / 32; ++kc)
        c = mfma16(frag_a(sD2, MLP_H, 1, 16 * rb, 32 * kc, lane), frag_b(P + OFF_W2, 1, MLP_H, 32 * kc, 16 * ib, lane),
                   c);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * rb + rq + q, i = 16 * ib + col;
        sD1[r * MLP_H + i] = bf16_round(sH1[r * MLP_H + i] > 0.f ? c[q] : 0.f);
      }
    }
  __syncthreads();
  // db1
  for (int i = lane; i < MLP_H; i += 64) {
    float acc = 0.f;
    for (int r = 0; r < BWD_ROWS; ++r) acc += sD1[r * MLP_H + i];
    g[OFF_B1 + i] = acc;
  }
  // dW1[k][i] = sum_r F[r][k] dH1[r][i]
  for (int kb = 0; kb < MLP_IN / 16; ++kb)
    for (int ib = 0; ib < MLP_H / 16; ++ib) {
      f32x4 c = {0.f, 0.f, 0.f, 0.f};
      c = mfma16(frag_a(sF, 1, MLP_IN, 16 * kb, 0, lane), frag_b(sD1, MLP_H, 1, 0, 16 * ib, lane), c);
#pragma unroll
      for (int q = 0; q < 4; ++q) g[OFF_W1 + (16 * kb + rq + q) * MLP_H + 16 * ib + col] = c[q];
    }
}

constexpr size_t BWD_LDS = sizeof(float) * (BWD_ROWS * MLP_IN + 4 * BWD_ROWS * MLP_H + BWD_ROWS);

// sum of the tile partials in tile order
__global__ void k_mlp_reduce(const float *__restrict__ gpart, const float *__restrict__ lpart, int ntiles,
                             float *__restrict__ grad, float *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MLP_NPARAM) {
    float acc = 0.f;
    for (int t = 0; t < ntiles; ++t) acc += gpart[(long long)t * MLP_NPARAM + p];
    grad[p] = acc;
  }
  if (p == 0 && loss) {
    float l = 0.f;
    for (int t = 0; t < ntiles; ++t) l += lpart[t];
    *loss = l;
  }
}

// Adam on the FP32 master weights (bias-corrected; step counts from 1)
__global__ void k_mlp_adam(float *__restrict__ P, float *__restrict__ m1, float *__restrict__ m2,
                           const float *__restrict__ grad, long long step, float lr, float beta1, float beta2,
                           float eps) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MLP_NPARAM) return;
  const float gr = grad[p];
  const float a = beta1 * m1[p] + (1.0f - beta1) * gr;
  const float b = beta2 * m2[p] + (1.0f - beta2) * gr * gr;
  m1[p] = a;
  m2[p] = b;
  const float c1 = 1.0f - powf(beta1, (float)step), c2 = 1.0f - powf(beta2, (float)step);
  const float mh = a / c1, vh = b / c2;
  P[p] = P[p] - lr * mh / (sqrtf(vh) + eps);
}

// ------------------------------------------------------ feature sign sums
// The features need D_jk = sum_i x_ij sgn(x_ik) and Zr_jk = sum_i |x_ij| [x_ik
// = 0] for every pair only to rank the columns (the exact solve computes its
// own in FP64), so they run on the BF16 matrix units.  Column j, scaled by the
// power of two 2^-(E_j) that brings its largest magnitude into [1, 2) (E_j its
// exponent), is split into BF16 parts h + l that carry 16 significant bits
// (|x - h - l| <= 2^-15 |x| after the scaling); the signs are exact in BF16.
//   D_jk  = 2^E_j sum_i (h_ij + l_ij) sgn(x_ik)       two products
//   Zr_jk = 2^E_j sum_i |h_ij| [x_ik = 0]              one product (terms >= 0:
//                                                     relative error 2^-8)
// with FP32 accumulation over the rows (error <= n 2^-24 of the sum of the
// terms' magnitudes).  Planes: bf16 [m][np], np = n rounded up to 32, rows
// past n zero in h and l (so they add nothing; their sign entries are +1).
constexpr int FSS_K = 32;            // rows per MFMA step
constexpr int FSS_T = 64;            // output block (j and k) of one wave

__host__ __device__ constexpr int64_t fss_rows(int64_t n) { return (n + FSS_K - 1) / FSS_K * FSS_K; }

__device__ __forceinline__ int col_exp(const ColInfo &c) { return c.nnz > 0 ? c.bemax - 1023 : 0; }

__global__ void __launch_bounds__(256)
k_feat_planes(const double *__restrict__ X, int n, int m, long long ld, int np, const ColInfo *__restrict__ ci,
              __bf16 *__restrict__ H, __bf16 *__restrict__ Lo, __bf16 *__restrict__ S) {
  // block b: column b / chunks, rows 256 (b % chunks) ...
  const int chunks = (np + 255) >> 8;
  const int j = blockIdx.x / chunks;
  const int i = (blockIdx.x % chunks) * 256 + threadIdx.x;
  if (j >= m || i >= np) return;
  const double x = i < n ? X[(long long)j * ld + i] : 0.0;
  const double xs = ldexp(x, -col_exp(ci[j]));
  const __bf16 h = (__bf16)(float)xs;
  const __bf16 l = (__bf16)(float)(xs - (double)(float)h);
  const long long o = (long long)j * np + i;
  H[o] = h;
  Lo[o] = l;
  S[o] = (__bf16)(i >= n ? 1.0f : (x > 0.0 ? 1.0f : (x < 0.0 ? -1.0f : 0.0f)));
}

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ bf16x8 ld_frag(const __bf16 *p) { return *(const bf16x8 *)p; }
__device__ __forceinline__ bf16x8 bits_and(bf16x8 v, uint32_t mask) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u &= mask;
  return __builtin_bit_cast(bf16x8, u);
}
// [s = 0] from a sign fragment: +-1 -> 0, 0 -> 1 (bit patterns 3F80, BF80, 0)
__device__ __forceinline__ bf16x8 zero_of_sign(bf16x8 v) {
  u32x4 u = __builtin_bit_cast(u32x4, v);
  u = (u & 0x7FFF7FFFu) ^ 0x3F803F80u;
  return __builtin_bit_cast(bf16x8, u);
}

// One wave per 64 x 64 block (j0, k0) of the m x m output; DZ[j m + k] =
// (D_jk, Zr_jk) in FP64.  Fragments straight from the planes (each lane reads
// 16 contiguous bytes of one column), the next step's prefetched.
__global__ void __launch_bounds__(256)
k_feat_signsum(const __bf16 *__restrict__ H, const __bf16 *__restrict__ Lo, const __bf16 *__restrict__ S, int m,
               int np, const ColInfo *__restrict__ ci, double2 *__restrict__ DZ) {
  const int lane = threadIdx.x & 63;
  const int tb = (m + FSS_T - 1) / FSS_T;
  const int t = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  if (t >= tb * tb) return;
  const int j0 = (t / tb) * FSS_T, k0 = (t % tb) * FSS_T;
  const int r = lane & 15, kq = 8 * (lane >> 4);
  // columns past m read column m - 1 (their results are not stored)
  long long oa[4], ob[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    oa[a] = (long long)min(j0 + 16 * a + r, m - 1) * np + kq;
    ob[a] = (long long)min(k0 + 16 * a + r, m - 1) * np + kq;
  }
  f32x4 accD[4][4], accZ[4][4];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      accD[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
      accZ[a][b] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  bf16x8 nh[4], nl[4], ns[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    nh[a] = ld_frag(H + oa[a]);
    nl[a] = ld_frag(Lo + oa[a]);
    ns[a] = ld_frag(S + ob[a]);
  }
  for (int i0 = 0; i0 < np; i0 += FSS_K) {
    bf16x8 fh[4], fl[4], fs[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
      fh[a] = nh[a];
      fl[a] = nl[a];
      fs[a] = ns[a];
    }
    if (i0 + FSS_K < np) {
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        nh[a] = ld_frag(H + oa[a] + i0 + FSS_K);
        nl[a] = ld_frag(Lo + oa[a] + i0 + FSS_K);
        ns[a] = ld_frag(S + ob[a] + i0 + FSS_K);
      }
    }
#pragma unroll
    for (int b = 0; b < 4; ++b) {
      const bf16x8 fz = zero_of_sign(fs[b]);
#pragma unroll
      for (int a = 0; a < 4; ++a) {
        accD[a][b] = mfma16(fh[a], fs[b], accD[a][b]);
        accD[a][b] = mfma16(fl[a], fs[b], accD[a][b]);
        accZ[a][b] = mfma16(bits_and(fh[a], 0x7FFF7FFFu), fz, accZ[a][b]);
      }
    }
  }
  // C layout: lane holds rows 4 (lane >> 4) + q (j), column lane & 15 (k)
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = j0 + 16 * a + 4 * (lane >> 4) + q;
      if (j >= m) continue;
      const int e = col_exp(ci[j]);
#pragma unroll
      for (int b = 0; b < 4; ++b) {
        const int k = k0 + 16 * b + r;
        if (k < m) DZ[(long long)j * m + k] = double2{ldexp((double)accD[a][b][q], e), ldexp((double)accZ[a][b][q], e)};
      }
    }
}

// ----------------------------------------------------------------- features
// Per column j, aggregates of the initial slopes s_jk = |D_jk| - Zr_jk - lambda
// of the segments (j, k != j) where 0 is not the minimiser (s_jk > 0): the
// objective is z_j = sum_k W_k - W_j + lambda - sum_k Delta_jk with
// Delta_jk = g_jk(0) - g_jk(v_k) >= 0, zero exactly when s_jk <= 0, and
// growing with s_jk.  agg[j] = (sum s, sum s^2 / W_k, sum s / W_k, count).
// One wave per column.
__global__ void k_slope_aggr(const double2 *__restrict__ DZ, const ColInfo *__restrict__ ci, int m, double lambda,
                             double *__restrict__ agg) {
  const int j = blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (j >= m) return;
  double s1 = 0.0, s2 = 0.0, s3 = 0.0, c = 0.0;
  for (int k = lane; k < m; k += 64) {
    if (k == j) continue;
    const double2 dz = DZ[(long long)j * m + k];
    const double sl = fabs(dz.x) - dz.y - lambda;
    if (sl > 0.0) {
      const double Wk = ci[k].W;
      s1 += sl;
      c += 1.0;
      if (Wk > 0.0) {
        s2 += sl * sl / Wk;
        s3 += sl / Wk;
      }
    }
  }
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) {
    s1 += __shfl_xor(s1, d);
    s2 += __shfl_xor(s2, d);
    s3 += __shfl_xor(s3, d);
    c += __shfl_xor(c, d);
  }
  if (lane == 0) {
    agg[4 * j + 0] = s1;
    agg[4 * j + 1] = s2;
    agg[4 * j + 2] = s3;
    agg[4 * j + 3] = c;
  }
}

constexpr int FEAT_Q = 5;   // quantities with statistics: W, and the four slope aggregates

// mean / standard deviation / max over the columns of W_j and of each
// aggregate: stats[3 q + (0, 1, 2)] (one workgroup of 256)
__global__ void k_feature_stats(const double *__restrict__ agg, int m, const ColInfo *__restrict__ ci,
                                double *__restrict__ stats) {
  __shared__ double sh[3][256];
  const int tid = threadIdx.x;
  for (int q = 0; q < FEAT_Q; ++q) {
    double mx = -1e300, sum = 0.0, sq = 0.0;
    for (int j = tid; j < m; j += blockDim.x) {
      const double v = q == 0 ? ci[j].W : agg[4 * j + q - 1];
      mx = fmax(mx, v);
      sum += v;
      sq += v * v;
    }
    sh[0][tid] = mx;
    sh[1][tid] = sum;
    sh[2][tid] = sq;
    __syncthreads();
    for (int st = blockDim.x >> 1; st > 0; st >>= 1) {
      if (tid < st) {
        sh[0][tid] = fmax(sh[0][tid], sh[0][tid + st]);
        sh[1][tid] += sh[1][tid + st];
        sh[2][tid] += sh[2][tid + st];
      }
      __syncthreads();
    }
    if (tid == 0) {
      const double mean = sh[1][0] / m;
      const double var = fmax(sh[2][0] / m - mean * mean, 0.0);
      stats[3 * q + 0] = mean;
      stats[3 * q + 1] = sqrt(var);
      stats[3 * q + 2] = sh[0][0];
    }
    __syncthreads();
  }
}

// the 32 features of column j (documented in the header)
__global__ void k_features(const double *__restrict__ agg, int m, int n, double lambda,
                           const ColInfo *__restrict__ ci, const double *__restrict__ stats, float *__restrict__ F) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= m) return;
  float f[MLP_IN];
#pragma unroll
  for (int q = 0; q < MLP_IN; ++q) f[q] = 0.f;
  const ColInfo c = ci[j];
  const double W = c.W, meanW = stats[0], sdW = stats[1], maxW = stats[2];
  f[0] = (float)(sdW > 0.0 ? (W - meanW) / sdW : 0.0);
  f[1] = (float)(sdW > 0.0 ? (W - maxW) / sdW : 0.0);
  f[2] = (float)(W > 0.0 && meanW > 0.0 ? log(W / meanW) : -30.0);
  f[3] = (float)c.zeros / (float)n;
  f[4] = (float)(W > 0.0 ? fmin(lambda / W, 10.0) : 10.0);
  f[5] = (float)(agg[4 * j + 3] / (double)(m > 1 ? m - 1 : 1));
#pragma unroll
  for (int q = 1; q < FEAT_Q; ++q) {
    const double v = agg[4 * j + q - 1], mean = stats[3 * q], sd = stats[3 * q + 1], mx = stats[3 * q + 2];
    f[4 + 2 * q] = (float)(sd > 0.0 ? (v - mean) / sd : 0.0);
    f[5 + 2 * q] = (float)(sd > 0.0 ? (v - mx) / sd : 0.0);
  }
  f[14] = (float)(W > 0.0 ? log1p(agg[4 * j] / W) : 0.0);
  f[15] = 1.0f;
#pragma unroll
  for (int q = 0; q < MLP_IN; ++q) F[(long long)j * MLP_IN + q] = f[q];
}

// ------------------------------------------------------------------- top-K
// K smallest scores (lowest index on ties), their list in increasing score,
// a candidate mask, and the margin between the first score left out and the
// best; fallback = (margin < threshold) or K >= m.
__global__ void k_topk(const float *__restrict__ score, int m, int K, double threshold, int *__restrict__ cand,
                       int *__restrict__ mask, int *__restrict__ fallback, float *__restrict__ margin_out) {
  __shared__ float sv[256];
  __shared__ int si[256];
  const int tid = threadIdx.x;
  for (int j = tid; j < m; j += blockDim.x) mask[j] = 0;
  __syncthreads();
  float best0 = 0.f, next = 0.f;
  for (int r = 0; r <= K && r < m; ++r) {
    float bv = 0.f;
    int bi = -1;
    for (int j = tid; j < m; j += blockDim.x) {
      if (mask[j]) continue;
      const float v = isnan(score[j]) ? INFINITY : score[j];
      if (bi < 0 || v < bv) { bv = v; bi = j; }
    }
    sv[tid] = bv;
    si[tid] = bi;
    __syncthreads();
    for (int s = blockDim.x >> 1; s > 0; s >>= 1) {
      if (tid < s) {
        const int oi = si[tid + s];
        const float ov = sv[tid + s];
        if (oi >= 0 && (si[tid] < 0 || ov < sv[tid] || (ov == sv[tid] && oi < si[tid]))) {
          sv[tid] = ov;
          si[tid] = oi;
        }
      }
      __syncthreads();
    }
    const int pick = si[0];
    const float pv = sv[0];
    __syncthreads();
    if (r == 0) best0 = pv;
    if (r < K) {
      if (tid == 0) {
        cand[r] = pick;
        mask[pick] = 1;
      }
    } else {
      next = pv;
    }
    __syncthreads();
  }
  if (tid == 0) {
    const float mg = (K < m) ? next - best0 : 0.f;
    *margin_out = mg;
    // a NaN margin (every score non-finite: inf - inf) or a non-finite best
    // score separates nothing: the exhaustive search decides
    *fallback = (K >= m || !((double)mg >= threshold) || !isfinite(best0)) ? 1 : 0;
  }
}

// The same selection for m <= TOPK_LDS_MAX by one sort in LDS (one workgroup
// of 1024): key = order-preserving bits of the score (NaN as +inf, -0 as +0)
// above the column index, so ascending keys are ascending scores with the
// lower index first on ties, as above; the candidates are the first K keys
// and the margin is score K minus score 0.
constexpr int TOPK_LDS_MAX = 8192;

__global__ void __launch_bounds__(1024)
k_topk_lds(const float *__restrict__ score, int m, int K, double threshold, int *__restrict__ cand,
           int *__restrict__ mask, int *__restrict__ fallback, float *__restrict__ margin_out) {
  __shared__ unsigned long long key[TOPK_LDS_MAX];
  const int tid = threadIdx.x;
  int N = 2;
  while (N < m) N <<= 1;
  auto score_key = [](float v) {
    v = isnan(v) ? INFINITY : v + 0.0f;
    const uint32_t u = __float_as_uint(v);
    return (uint32_t)((u >> 31) ? ~u : (u | 0x80000000u));
  };
  auto key_score = [](uint32_t k) { return __uint_as_float((k >> 31) ? (k & 0x7FFFFFFFu) : ~k); };
  for (int j = tid; j < N; j += blockDim.x) {
    key[j] = j < m ? ((unsigned long long)score_key(score[j]) << 32) | (uint32_t)j : ~0ull;
    if (j < m) mask[j] = 0;
  }
  __syncthreads();
  for (int k = 2; k <= N; k <<= 1)
    for (int h = k >> 1; h > 0; h >>= 1) {
      for (int i = tid; i < N; i += blockDim.x) {
        const int o = i ^ h;
        if (o > i) {
          const unsigned long long a = key[i], b = key[o];
          if ((a > b) == ((i & k) == 0)) {
            key[i] = b;
            key[o] = a;
          }
        }
      }
      __syncthreads();
    }
  const int kk = K < m ? K : m;
  for (int r = tid; r < kk; r += blockDim.x) {
    const int j = (int)(uint32_t)key[r];
    cand[r] = j;
    mask[j] = 1;
  }
  if (tid == 0) {
    const float best0 = key_score((uint32_t)(key[0] >> 32));
    const float mg = (K < m) ? key_score((uint32_t)(key[K] >> 32)) - best0 : 0.f;
    *margin_out = mg;
    *fallback = (K >= m || !((double)mg >= threshold) || !isfinite(best0)) ? 1 : 0;
  }
}

// ------------------------------------------------------- training matrices
// Counter-based generator: Philox-4x32-10 (Salmon, Moraes, Dror, Shaw,
// "Parallel random numbers: as easy as 1, 2, 3", SC 2011), written from its
// published definition: ten rounds of two 32x32->64 multiplications with
// the round keys bumped by the Weyl constants.
struct PhiloxKey {
  uint32_t k0, k1;
};
__device__ __forceinline__ uint4 philox4x32(uint4 c, PhiloxKey k) {
  constexpr uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u, W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t hi0 = __umulhi(M0, c.x), lo0 = M0 * c.x;
    const uint32_t hi1 = __umulhi(M1, c.z), lo1 = M1 * c.z;
    c = make_uint4(hi1 ^ c.y ^ k.k0, lo1, hi0 ^ c.w ^ k.k1, lo0);
    k.k0 += W0;
    k.k1 += W1;
  }
  return c;
}
// uniform in (0, 1) from 32 random bits; standard normal by Box-Muller
__device__ __forceinline__ double unit_open(uint32_t u) { return ((double)u + 0.5) * 0x1p-32; }
__device__ __forceinline__ double normal_of(uint32_t a, uint32_t b) {
  return sqrt(-2.0 * log(unit_open(a))) * cos(6.283185307179586 * unit_open(b));
}

// One training matrix n x m (column-major, ld = n) of the rank-one recipe:
// x_ik = u_i l_k + e_ik with u_i ~ N(0,1), l_k ~ U[-1,1] on a random 10% of
// the columns (0 elsewhere), e_ik ~ Laplace(0, 0.1) by inversion; a random
// 10% of the rows replaced by 20 N(0,1); 1% of the entries set to +0.0.
// Every random choice is an independent Bernoulli draw keyed by (seed,
// example, row, column), so no permutation is needed.
__global__ void k_gen_training(double *__restrict__ X, int n, int m, PhiloxKey key) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * m) return;
  const int k = (int)(e / n), i = (int)(e % n);
  const uint4 rr = philox4x32(make_uint4((uint32_t)i, 0xFFFFFFFFu, 1u, 0u), key);   // row draws
  const uint4 rc = philox4x32(make_uint4(0xFFFFFFFFu, (uint32_t)k, 2u, 0u), key);   // column draws
  const uint4 re = philox4x32(make_uint4((uint32_t)i, (uint32_t)k, 3u, 0u), key);   // entry draws
  const double u = normal_of(rr.x, rr.y);
  const bool outlier_row = unit_open(rr.z) < 0.1;
  const double l = unit_open(rc.x) < 0.1 ? 2.0 * unit_open(rc.y) - 1.0 : 0.0;
  double x;
  if (outlier_row) {
    x = 20.0 * normal_of(re.x, re.y);
  } else {
    const double h = unit_open(re.x) - 0.5;
    const double lap = -0.1 * (h < 0.0 ? -1.0 : 1.0) * log1p(-2.0 * fabs(h));
    x = u * l + lap;
  }
  if (unit_open(re.z) < 0.01) x = 0.0;
  X[(long long)k * n + i] = x;
}

// max over the columns of the column mass (one workgroup of 256)
__global__ void k_max_mass(const ColInfo *__restrict__ ci, int m, double *__restrict__ out) {
  __shared__ double sh[256];
  double mx = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) mx = fmax(mx, ci[j].W);
  sh[threadIdx.x] = mx;
  __syncthreads();
  for (int st = blockDim.x >> 1; st > 0; st >>= 1) {
    if (threadIdx.x < st) sh[threadIdx.x] = fmax(sh[threadIdx.x], sh[threadIdx.x + st]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *out = sh[0];
}

// training targets y_j = (z_j - min z) / (mean z - min z) (0 when the
// objectives are all equal); one workgroup of 256
__global__ void k_targets(const double *__restrict__ z, int m, float *__restrict__ y) {
  __shared__ double smin[256], ssum[256];
  double mn = 1e308, sum = 0.0;
  for (int j = threadIdx.x; j < m; j += blockDim.x) {
    mn = fmin(mn, z[j]);
    sum += z[j];
  }
  smin[threadIdx.x] = mn;
  ssum[threadIdx.x] = sum;
  __syncthreads();
  for (int st = blockDim.x >> 1; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + st]);
      ssum[threadIdx.x] += ssum[threadIdx.x + st];
    }
    __syncthreads();
  }
  const double lo = smin[0], span = ssum[0] / m - lo;
  for (int j = threadIdx.x; j < m; j += blockDim.x) y[j] = (float)(span > 0.0 ? (z[j] - lo) / span : 0.0);
}
