// peak_kernels.h -- microbenchmarks that measure the MI355X ceilings the
// roofline figures divide by: HBM copy bandwidth, LDS read bandwidth, FP64
// FMA issue on the VALU, and the FP64 and BF16 matrix (MFMA) rates.  Every
// kernel keeps its results live (a data-dependent store) so nothing is
// optimised away, and runs far more work than launch overhead.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// HBM: a streaming copy, 16 bytes per thread and step, grid-stride.
__global__ void __launch_bounds__(256) k_peak_copy(const double2 *__restrict__ src, double2 *__restrict__ dst,
                                                   long long n) {
  const long long stride = (long long)gridDim.x * blockDim.x;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = src[i];
}

// LDS: every thread reads 16 bytes per step from a 16 KB block (four
// independent streams, conflict-free consecutive addresses), ITER steps.
constexpr int PEAK_LDS_ITER = 4096;
__global__ void __launch_bounds__(256) k_peak_lds(unsigned *__restrict__ sink) {
  __shared__ uint4 buf[1024];
  const int tid = threadIdx.x;
  for (int e = tid; e < 1024; e += 256) buf[e] = make_uint4(e, e + 1, e + 2, e + 3);
  __syncthreads();
  uint4 acc[4] = {};
#pragma unroll 4
  for (int it = 0; it < PEAK_LDS_ITER; ++it) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const uint4 v = buf[(tid + 256 * q + it) & 1023];
      acc[q].x ^= v.x;
      acc[q].y ^= v.y;
      acc[q].z ^= v.z;
      acc[q].w ^= v.w;
    }
  }
  unsigned r = 0;
#pragma unroll
  for (int q = 0; q < 4; ++q) r ^= acc[q].x ^ acc[q].y ^ acc[q].z ^ acc[q].w;
  if (r == 0x9E3779B9u) sink[blockIdx.x * 256 + tid] = r;
}

// FP64 VALU: 8 independent FMA chains per thread, ITER steps (2 flops each).
constexpr int PEAK_FMA_ITER = 2048;
__global__ void __launch_bounds__(256) k_peak_fma(double *__restrict__ sink, double a, double b) {
  double x[8];
#pragma unroll
  for (int c = 0; c < 8; ++c) x[c] = threadIdx.x * 1e-3 + c;
  for (int it = 0; it < PEAK_FMA_ITER; ++it) {
#pragma unroll
    for (int c = 0; c < 8; ++c) x[c] = fma(x[c], a, b);
  }
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < 8; ++c) r += x[c];
  if (r == 1234.5) sink[blockIdx.x * 256 + threadIdx.x] = r;
}

// FP64 matrix: v_mfma_f64_16x16x4f64 (2 x 16 x 16 x 4 = 2048 flops per wave
// instruction), four independent accumulators per wave.
typedef double peak_f64x4 __attribute__((ext_vector_type(4)));
constexpr int PEAK_MFMA_ITER = 1024;
__global__ void __launch_bounds__(256) k_peak_mfma_f64(double *__restrict__ sink, double a) {
  peak_f64x4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = (peak_f64x4){0.0, 0.0, 0.0, 0.0};
  const double b = a * (threadIdx.x & 63);
  for (int it = 0; it < PEAK_MFMA_ITER; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc[c], 0, 0, 0);
  }
  double r = 0.0;
#pragma unroll
  for (int c = 0; c < 4; ++c) r += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (r == 1234.5) sink[blockIdx.x * 256 + threadIdx.x] = r;
}

// BF16 matrix: v_mfma_f32_16x16x32_bf16 (2 x 16 x 16 x 32 = 16384 flops per
// wave instruction), four independent accumulators per wave.
typedef __bf16 peak_bf16x8 __attribute__((ext_vector_type(8)));
typedef float peak_f32x4 __attribute__((ext_vector_type(4)));
__global__ void __launch_bounds__(256) k_peak_mfma_bf16(float *__restrict__ sink, float a) {
  peak_bf16x8 va, vb;
#pragma unroll
  for (int q = 0; q < 8; ++q) {
    va[q] = (__bf16)(a * (q + 1));
    vb[q] = (__bf16)(a * (threadIdx.x & 7));
  }
  peak_f32x4 acc[4];
#pragma unroll
  for (int c = 0; c < 4; ++c) acc[c] = (peak_f32x4){0.f, 0.f, 0.f, 0.f};
  for (int it = 0; it < PEAK_MFMA_ITER; ++it) {
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(va, vb, acc[c], 0, 0, 0);
  }
  float r = 0.f;
#pragma unroll
  for (int c = 0; c < 4; ++c) r += acc[c][0] + acc[c][1] + acc[c][2] + acc[c][3];
  if (r == 1234.5f) sink[blockIdx.x * 256 + threadIdx.x] = r;
}
