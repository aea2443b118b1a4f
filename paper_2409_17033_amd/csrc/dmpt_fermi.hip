// Elementwise and reduction kernels of the finite-temperature path (Sec. V.B).
// The products of the recursion run on k_gemm_nt (FP32 MFMA); these kernels
// form the start matrices, linear combinations, symmetrisations and traces.
#include <hip/hip_runtime.h>

#include "dmpt_fermi.h"

namespace dmpt {

namespace {

__device__ __forceinline__ double wave_sum64(double v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// One 64 x 64 output block per workgroup; the block and its transpose are
// staged through LDS so both are read row-wise.
__global__ __launch_bounds__(256) void k_fermi_start(const float* src, int n, int n_pad, double scale, double shift,
                                                     float* dst) {
  __shared__ float t[64][65];
  __shared__ float tt[64][65];
  const int bi = blockIdx.y, bj = blockIdx.x;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gi = bi * 64 + r, gj = bj * 64 + c;
    const int hi = bj * 64 + r, hj = bi * 64 + c;
    t[r][c] = (gi < n && gj < n) ? src[(size_t)gi * n + gj] : 0.0f;
    tt[r][c] = (hi < n && hj < n) ? src[(size_t)hi * n + hj] : 0.0f;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const int gi = bi * 64 + r, gj = bj * 64 + c;
    double v = 0.5 * ((double)t[r][c] + (double)tt[c][r]);
    if (gi == gj && gi < n) v -= shift;
    dst[(size_t)gi * n_pad + gj] = (gi < n && gj < n) ? (float)(scale * v) : 0.0f;
  }
}

// One row per block iteration (coalesced, no index division).
__global__ __launch_bounds__(256) void k_axpby(float* z, const float* x, float a, const float* y, float b, float d,
                                               int nd, int n_pad) {
  for (int i = blockIdx.x; i < n_pad; i += gridDim.x) {
    const size_t row = (size_t)i * n_pad;
    for (int j = threadIdx.x; j < n_pad; j += 256) {
      float v = a * x[row + j];
      if (y) v += b * y[row + j];
      if (i == j && i < nd) v += d;
      z[row + j] = v;
    }
  }
}

__global__ __launch_bounds__(256) void k_symm(const float* in, float alpha, const float* x, float beta, float* out,
                                              int n_pad) {
  __shared__ float t[64][65];
  __shared__ float tt[64][65];
  const int bi = blockIdx.y, bj = blockIdx.x;
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    t[r][c] = in[(size_t)(bi * 64 + r) * n_pad + bj * 64 + c];
    tt[r][c] = in[(size_t)(bj * 64 + r) * n_pad + bi * 64 + c];
  }
  __syncthreads();
  for (int e = threadIdx.x; e < 64 * 64; e += 256) {
    const int r = e >> 6, c = e & 63;
    const size_t o = (size_t)(bi * 64 + r) * n_pad + bj * 64 + c;
    float v = alpha * (t[r][c] + tt[c][r]);
    if (x) v += beta * x[o];
    out[o] = v;
  }
}

// Block b sums rows 64b .. 64b + 63 of the leading n x n block, one wave per
// 16 rows, in a fixed order.
// (Tr M, ||M||_F^2) over the leading n x n block of an n_pad-strided matrix:
// one wave per row, 16-byte loads when the rows allow it (n % 4 == 0 and M
// 16-byte aligned), two accumulators per lane; block b adds its four rows in
// order into part[2b], part[2b + 1] (the host sums the blocks in order).
__global__ __launch_bounds__(256) void k_trace_sq(const float* m, int n, int n_pad, double* part) {
  __shared__ double s_tr[4], s_sq[4];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int i = blockIdx.x * 4 + wave;
  double tr = 0.0, sq0 = 0.0, sq1 = 0.0;
  if (i < n) {
    const float* row = m + (size_t)i * n_pad;
    if ((n & 3) == 0 && ((uintptr_t)m & 15) == 0) {
      typedef float f4 __attribute__((ext_vector_type(4)));
      const f4* row4 = (const f4*)row;
      const int n4 = n >> 2;
      int q = lane;
      for (; q + 64 < n4; q += 128) {
        const f4 x0 = row4[q], x1 = row4[q + 64];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          sq0 += (double)x0[e] * (double)x0[e];
          sq1 += (double)x1[e] * (double)x1[e];
        }
      }
      if (q < n4) {
        const f4 x0 = row4[q];
#pragma unroll
        for (int e = 0; e < 4; ++e) sq0 += (double)x0[e] * (double)x0[e];
      }
    } else {
      for (int j = lane; j < n; j += 64) {
        const double v = row[j];
        sq0 += v * v;
      }
    }
    if (lane == 0) tr = row[i];
  }
  const double sq = wave_sum64(sq0 + sq1);
  if (lane == 0) {
    s_tr[wave] = tr;
    s_sq[wave] = sq;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = s_tr[0] + s_tr[1] + s_tr[2] + s_tr[3];
    part[2 * blockIdx.x + 1] = s_sq[0] + s_sq[1] + s_sq[2] + s_sq[3];
  }
}

}  // namespace

hipError_t launch_fermi_start(const float* src, int n, int n_pad, double scale, double shift, float* dst,
                              hipStream_t s) {
  const int nb = n_pad / 64;
  hipLaunchKernelGGL(k_fermi_start, dim3(nb, nb), dim3(256), 0, s, src, n, n_pad, scale, shift, dst);
  return hipGetLastError();
}

hipError_t launch_axpby(float* z, const float* x, float a, const float* y, float b, float d, int nd, int n_pad,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_axpby, dim3(2048), dim3(256), 0, s, z, x, a, y, b, d, nd, n_pad);
  return hipGetLastError();
}

hipError_t launch_symm(const float* in, float alpha, const float* x, float beta, float* out, int n_pad,
                       hipStream_t s) {
  const int nb = n_pad / 64;
  hipLaunchKernelGGL(k_symm, dim3(nb, nb), dim3(256), 0, s, in, alpha, x, beta, out, n_pad);
  return hipGetLastError();
}

int trace_sq_blocks(int n_pad) { return n_pad / 4; }   // one row per wave, four per block

hipError_t launch_trace_sq(const float* m, int n, int n_pad, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_trace_sq, dim3(trace_sq_blocks(n_pad)), dim3(256), 0, s, m, n, n_pad, part);
  return hipGetLastError();
}

}  // namespace dmpt
