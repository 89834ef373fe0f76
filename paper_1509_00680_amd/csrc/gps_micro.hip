// Measurement kernels behind three design decisions of the FFT passes
// (libgps_micro.so, loaded only by the benchmark; not part of include/gps.h):
//  * the issue rate of the register FFT codelets: one 16-point DFT per lane,
//    applied repeatedly to values held in registers (no memory traffic);
//  * the same DFT as a dense real GEMM on the matrix cores
//    (v_mfma_f32_16x16x4_f32): a 16-point complex DFT of 16 pencils is the
//    32 x 32 real matrix [[C, S], [-S, C]] (C = cos, S = sin of 2 pi n k/16)
//    times the 32 x 16 matrix of the pencils' real and imaginary parts, i.e.
//    16 MFMA instructions per 16 pencils.  One kernel computes that product
//    once and writes it (so the host can check it against a library FFT); the
//    timing kernel issues the same 16 MFMAs per 16 pencils with register
//    operands only, which bounds any MFMA form of the stage from above;
//  * a pointwise stream of 5 reads and 2 writes per point (the shape of the
//    PCG vector work) over XCD-contiguous chunks, the floor of such a pass.
#include <hip/hip_runtime.h>

#include "gps_fft_reg.h"

namespace {

using gps::cplx;
typedef float v4f __attribute__((ext_vector_type(4)));

__global__ __launch_bounds__(256) void k_codelet16(int reps, float* out) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  cplx<float> x[16];
#pragma unroll
  for (int j = 0; j < 16; ++j) x[j] = gps::cmk(float(t & 7) + 0.125f * j, 0.5f - 0.0625f * j);
  for (int r = 0; r < reps; ++r) {
    gps::reg_fft<float, false, 16>(x);
#pragma unroll
    for (int j = 0; j < 16; ++j) x[j] = gps::cscale(x[j], 0.25f);   // |DFT| grows by 4
  }
  float s = 0.f;
#pragma unroll
  for (int j = 0; j < 16; ++j) s += x[j].x + x[j].y;
  out[t] = s;
}

// Entry (row, col) of the 32 x 32 real DFT matrix.
__device__ __forceinline__ float dft_real(int row, int col) {
  const int k = row & 15, n = col & 15;
  float s, c;
  sincospif(float((n * k) & 15) / 8.0f, &s, &c);    // angle 2 pi n k / 16
  if (row < 16) return col < 16 ? c : s;
  return col < 16 ? -s : c;
}

// One wavefront: y (32 x 16, row-major) = DFT matrix x (32 x 16), i.e. the
// 16-point DFTs of 16 pencils, x[k][p] = Re (k < 16) / Im (k >= 16) of pencil
// p's element k mod 16.  Operand layout of v_mfma_f32_16x16x4_f32: lane l
// supplies A[l mod 16][l / 16] and B[l / 16][l mod 16]; its accumulator holds
// D[4 (l / 16) + i][l mod 16], i = 0..3.
__global__ __launch_bounds__(64) void k_mfma_dft16_check(const float* __restrict__ x,
                                                         float* __restrict__ y) {
  const int l = threadIdx.x;
  const int lr = l & 15, lk = l >> 4;
#pragma unroll
  for (int T = 0; T < 2; ++T) {
    v4f d = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      const float a = dft_real(16 * T + lr, 4 * s + lk);
      const float b = x[(4 * s + lk) * 16 + lr];
      d = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, d, 0, 0, 0);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i) y[(16 * T + 4 * lk + i) * 16 + lr] = d[i];
  }
}

// Throughput of the GEMM form: per repetition each wavefront issues the 16
// MFMAs of one 16-pencil DFT (two independent accumulator chains), operands
// in registers.
__global__ __launch_bounds__(256) void k_mfma_dft16_rate(int reps, float* out) {
  const int l = threadIdx.x & 63;
  float a[16], b[8];
#pragma unroll
  for (int j = 0; j < 16; ++j) a[j] = 0.001f * float((l + 3 * j) & 31);
#pragma unroll
  for (int j = 0; j < 8; ++j) b[j] = 0.002f * float((l + 5 * j) & 31);
  v4f d0 = {0.f, 0.f, 0.f, 0.f}, d1 = {0.f, 0.f, 0.f, 0.f};
  for (int r = 0; r < reps; ++r) {
#pragma unroll
    for (int s = 0; s < 8; ++s) {
      d0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[s], b[s], d0, 0, 0, 0);
      d1 = __builtin_amdgcn_mfma_f32_16x16x4f32(a[8 + s], b[s], d1, 0, 0, 0);
    }
  }
  out[blockIdx.x * blockDim.x + threadIdx.x] = d0[0] + d0[1] + d0[2] + d0[3] + d1[0] + d1[1] +
                                               d1[2] + d1[3];
}

// f = a + b * c, g = d - e * c over n points, 8 per thread, XCD-contiguous chunks.
__global__ __launch_bounds__(256) void k_stream5(long long n, const float* __restrict__ a,
                                                 const float* __restrict__ b,
                                                 const float* __restrict__ c,
                                                 const float* __restrict__ d,
                                                 const float* __restrict__ e,
                                                 float* __restrict__ f, float* __restrict__ g) {
  const long long base =
      (long long)gps::xcd_tile(blockIdx.x, gridDim.x) * 256 * 8 + threadIdx.x;
#pragma unroll
  for (int j = 0; j < 8; ++j) {
    const long long i = base + (long long)j * 256;
    if (i < n) {
      const float cv = c[i];
      f[i] = a[i] + b[i] * cv;
      g[i] = d[i] - e[i] * cv;
    }
  }
}

}  // namespace

extern "C" {

// All calls enqueue on `stream` (hipStream_t) and return at once; 0 on
// success, else the hipError_t of the launch.
int micro_codelet16(int blocks, int reps, float* out, void* stream) {
  hipLaunchKernelGGL(k_codelet16, dim3(blocks), dim3(256), 0, (hipStream_t)stream, reps, out);
  return (int)hipGetLastError();
}

int micro_mfma_dft16_check(const float* x, float* y, void* stream) {
  hipLaunchKernelGGL(k_mfma_dft16_check, dim3(1), dim3(64), 0, (hipStream_t)stream, x, y);
  return (int)hipGetLastError();
}

int micro_mfma_dft16_rate(int blocks, int reps, float* out, void* stream) {
  hipLaunchKernelGGL(k_mfma_dft16_rate, dim3(blocks), dim3(256), 0, (hipStream_t)stream, reps,
                     out);
  return (int)hipGetLastError();
}

int micro_stream5(long long n, const float* a, const float* b, const float* c, const float* d,
                  const float* e, float* f, float* g, void* stream) {
  const int groups = (int)((n + 256 * 8 - 1) / (256 * 8));
  hipLaunchKernelGGL(k_stream5, dim3(groups), dim3(256), 0, (hipStream_t)stream, n, a, b, c, d,
                     e, f, g);
  return (int)hipGetLastError();
}

}  // extern "C"
