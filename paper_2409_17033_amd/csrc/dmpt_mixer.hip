// gfx950 kernels of the self-consistent response loop (Eq. CP_SCF): the
// vector steps on the diagonal state v = diag(chi'), and the learned mixer.
//
// The mixer network is applied site by site with shared weights: for a
// state vector x in R^n, site i sees z_i = [x_{i-w} .. x_{i+w}, e_{i-w} ..
// e_{i+w}, U_i] with e the on-site energies (k = 4w + 3 features, zeros
// beyond the ends) and outputs
//   y_i = w2 . tanh(W1 z_i + b1) + b2          (hidden width h).
// Parameters (FP32 masters and the BF16 copy alike): [W1 (h x k, row-major) |
// b1 (h) | w2 (h) | b2 (1)].  Training: MSE loss, Adam (Kingma & Ba, 2015).
// Shapes are small next to the SP2 products (B n ~ 1e4-1e5 site rows,
// k ~ 66, h = 256), so the products use one LDS-tiled FP32 kernel with an
// optional deterministic split over K; weights are read as BF16 and widened.
#include <hip/hip_runtime.h>

#include <cmath>

#include "dmpt_internal.h"
#include "dmpt_scf.h"

namespace dmpt {

namespace {

__device__ __forceinline__ float ld(const float* p, size_t i) { return p[i]; }
__device__ __forceinline__ float ld(const uint16_t* p, size_t i) {
  return __builtin_bit_cast(float, ((unsigned int)p[i]) << 16);
}
__device__ __forceinline__ uint16_t to_bf16(float x) { return __builtin_bit_cast(uint16_t, (__bf16)x); }

constexpr int GT = 32;   // output tile edge; 256 threads, 4 outputs each

// C_z[m][c] = sum_{k in split z} a(m, k) b(k, c), C_z = C + z * zstride
//   a(m, k) = TRA ? A[k * lda + m] : A[m * lda + k]
//   b(k, c) = TRB ? B[c * ldb + k] : B[k * ldb + c]
template <class TA, class TB, bool TRA, bool TRB>
__global__ __launch_bounds__(256) void k_gemm(const TA* A, int lda, const TB* B, int ldb, float* C, int ldc,
                                              size_t zstride, int M, int N, int K, int kc) {
  __shared__ float sa[GT][GT + 1];
  __shared__ float sb[GT][GT + 1];
  const int t = threadIdx.x;
  const int m0 = blockIdx.y * GT, c0 = blockIdx.x * GT;
  const int kbeg = blockIdx.z * kc, kend = min(K, kbeg + kc);
  const int tr = t / 8, tc = (t % 8) * 4;   // this thread: row tr, columns tc..tc+3
  float acc[4] = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = kbeg; k0 < kend; k0 += GT) {
    for (int e = t; e < GT * GT; e += 256) {
      const int i = e / GT, j = e % GT;
      // sa[i][j] = a(m0 + i, k0 + j); sb[i][j] = b(k0 + i, c0 + j)
      const int am = m0 + i, ak = k0 + j;
      sa[i][j] = (am < M && ak < kend) ? ld(A, TRA ? (size_t)ak * lda + am : (size_t)am * lda + ak) : 0.f;
      const int bk = k0 + i, bc = c0 + j;
      sb[i][j] = (bk < kend && bc < N) ? ld(B, TRB ? (size_t)bc * ldb + bk : (size_t)bk * ldb + bc) : 0.f;
    }
    __syncthreads();
#pragma unroll 8
    for (int k = 0; k < GT; ++k) {
      const float av = sa[tr][k];
#pragma unroll
      for (int q = 0; q < 4; ++q) acc[q] += av * sb[k][tc + q];
    }
    __syncthreads();
  }
  float* cz = C + blockIdx.z * zstride;
  const int m = m0 + tr;
  if (m < M)
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (c0 + tc + q < N) cz[(size_t)m * ldc + c0 + tc + q] = acc[q];
}

// C[e] = sum_z P[z][e] for e < count (fixed order)
__global__ void k_sum_splits(const float* part, int splits, size_t count, float* c) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= count) return;
  float acc = 0.f;
  for (int z = 0; z < splits; ++z) acc += part[(size_t)z * count + e];
  c[e] = acc;
}

unsigned blocks(size_t total, unsigned per) { return (unsigned)((total + per - 1) / per); }

template <class TA, class TB, bool TRA, bool TRB>
hipError_t gemm(const TA* A, int lda, const TB* B, int ldb, float* C, int ldc, int M, int N, int K,
                hipStream_t s) {
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, 1);
  hipLaunchKernelGGL((k_gemm<TA, TB, TRA, TRB>), grid, dim3(256), 0, s, A, lda, B, ldb, C, ldc, (size_t)0, M, N,
                     K, K);
  return hipGetLastError();
}

// Long-K products (weight gradients over all site rows): K split into
// `splits` ranges, partial products into `scratch` (splits x M x N), then
// summed in a fixed order into the dense C (ldc = N).
constexpr int kSplits = 64;
template <class TA, class TB, bool TRA, bool TRB>
hipError_t gemm_splitk(const TA* A, int lda, const TB* B, int ldb, float* C, int M, int N, int K, float* scratch,
                       hipStream_t s) {
  const int kc = ((K + kSplits - 1) / kSplits + GT - 1) / GT * GT;
  const int splits = (K + kc - 1) / kc;
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT, splits);
  hipLaunchKernelGGL((k_gemm<TA, TB, TRA, TRB>), grid, dim3(256), 0, s, A, lda, B, ldb, scratch, N,
                     (size_t)M * N, M, N, K, kc);
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks((size_t)M * N, 256)), dim3(256), 0, s, scratch, splits,
                     (size_t)M * N, C);
  return hipGetLastError();
}

// Column sums of a rows x c matrix: chunk z of the rows into part[z][c]
// (then k_sum_splits over the chunks, fixed order).
__global__ void k_colsum_part(const float* m, size_t rows, int c, size_t chunk, float* part) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= c) return;
  const size_t r0 = (size_t)blockIdx.y * chunk, r1 = r0 + chunk < rows ? r0 + chunk : rows;
  float acc = 0.f;
  for (size_t r = r0; r < r1; ++r) acc += m[r * c + j];
  part[(size_t)blockIdx.y * c + j] = acc;
}

hipError_t colsum(const float* m, size_t rows, int c, float* out, float* scratch, hipStream_t s) {
  const size_t chunk = (rows + kSplits - 1) / kSplits;
  const int nchunk = (int)((rows + chunk - 1) / chunk);
  hipLaunchKernelGGL(k_colsum_part, dim3(blocks(c, 256), nchunk), dim3(256), 0, s, m, rows, c, chunk, scratch);
  hipLaunchKernelGGL(k_sum_splits, dim3(blocks(c, 256)), dim3(256), 0, s, scratch, nchunk, (size_t)c, out);
  return hipGetLastError();
}

// Z ((B n) x k): rows (b, i) = [x_b,i-w .. x_b,i+w, en_i-w .. en_i+w, U_i]
__global__ void k_site_inputs(const float* x, const float* u, const float* en, int B, int n, int w, float* z) {
  const int m = 2 * w + 1, k = 2 * m + 1;
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)B * n * k) return;
  const size_t row = e / k;
  const int f = (int)(e % k);
  const int b = (int)(row / n), i = (int)(row % n);
  float v;
  if (f == k - 1) {
    v = u[i];
  } else if (f < m) {
    const int j = i + f - w;
    v = (j >= 0 && j < n) ? x[(size_t)b * n + j] : 0.0f;
  } else {
    const int j = i + (f - m) - w;
    v = (j >= 0 && j < n) ? en[j] : 0.0f;
  }
  z[e] = v;
}

__global__ void k_diag(const float* m, int n, float* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = m[(size_t)i * n + i];
}

// Z (rows x h) += b1, then A = tanh(Z) in place.
__global__ void k_bias_tanh(float* z, const uint16_t* b1, size_t rows, int h) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < rows * h) z[e] = tanhf(z[e] + ld(b1, e % h));
}

// y (rows) += b2
__global__ void k_bias1(float* y, const uint16_t* b2, size_t rows) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < rows) y[e] += ld(b2, 0);
}

// dY = 2 (Y - T) / m in place of Y; per-block FP64 partials of sum (Y - T)^2.
__global__ __launch_bounds__(256) void k_mse(float* y, const float* t, size_t m, double* part) {
  __shared__ double red[4];
  const double scale = 2.0 / (double)m;
  double acc = 0.0;
  for (size_t e = (size_t)blockIdx.x * 256 + threadIdx.x; e < m; e += (size_t)gridDim.x * 256) {
    const double r = (double)y[e] - (double)t[e];
    acc += r * r;
    y[e] = (float)(scale * r);
  }
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// loss = sum(part) * inv, written to out[idx] (fixed order, one block).
__global__ void k_loss_final(const double* part, int nblk, double inv, double* out, int idx) {
  double acc = 0.0;
  for (int b = threadIdx.x; b < nblk; b += 64) acc += part[b];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (threadIdx.x == 0) out[idx] = acc * inv;
}

// dZ = dA * (1 - A^2) in place of dA (A = tanh(Z) kept from the forward pass).
__global__ void k_tanh_back(float* da, const float* a, size_t total) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) da[e] *= 1.0f - a[e] * a[e];
}

// Adam on the FP32 masters; refreshes the BF16 copy.
__global__ void k_adam(float* p, uint16_t* p16, float* m, float* v, const float* g, size_t count, float lr,
                       float beta1, float beta2, float eps, float c1, float c2) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const float gi = g[i];
  const float mi = beta1 * m[i] + (1.0f - beta1) * gi;
  const float vi = beta2 * v[i] + (1.0f - beta2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi * c1) / (sqrtf(vi * c2) + eps);
  p[i] = pi;
  p16[i] = to_bf16(pi);
}

// Initial weights: W ~ U(-r, r) with r = sqrt(6 / (fan_in + fan_out)) (Glorot),
// biases 0; the uniform numbers come from splitmix64 of (seed, index).
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}
__global__ void k_init_params(float* p, uint16_t* p16, int k, int h, uint64_t seed) {
  const size_t count = (size_t)h * k + 2 * h + 1;
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const size_t w1 = (size_t)h * k, b1 = w1 + h, w2 = b1 + h;
  float val = 0.0f;
  if (i < w1 || (i >= b1 && i < w2)) {
    const double u = (double)(splitmix64(seed * 0x100000001B3ull + i) >> 11) * (1.0 / 9007199254740992.0);
    const double r = i < w1 ? sqrt(6.0 / (double)(k + h)) : sqrt(6.0 / (double)(h + 1));
    val = (float)((2.0 * u - 1.0) * r);
  }
  p[i] = val;
  p16[i] = to_bf16(val);
}

}  // namespace

size_t mixer_param_count(int w, int h) { return (size_t)h * mixer_features(w) + 2 * h + 1; }

hipError_t mixer_diag(const float* m, int n, float* out, hipStream_t s) {
  hipLaunchKernelGGL(k_diag, dim3(blocks(n, 256)), dim3(256), 0, s, m, n, out);
  return hipGetLastError();
}

size_t mixer_scratch_floats(int n, int w, int h, int B) {
  const size_t rows = (size_t)B * n, k = mixer_features(w);
  // z, a, y, da, split partials of the weight gradients
  return rows * k + rows * h + rows + rows * h + (size_t)kSplits * (h * k + h + 1);
}

// forward: y (B x n) for states x (B x n).  scratch: mixer_scratch_floats.
hipError_t mixer_forward(const uint16_t* p16, int w, int h, const float* u, const float* en, int n, const float* x,
                         int B, float* y, float* scratch, hipStream_t s) {
  const int k = mixer_features(w);
  const size_t rows = (size_t)B * n;
  const uint16_t* w1 = p16;
  const uint16_t* b1 = w1 + (size_t)h * k;
  const uint16_t* w2 = b1 + h;
  const uint16_t* b2 = w2 + h;
  float* z = scratch;
  float* a = z + rows * k;
  hipLaunchKernelGGL(k_site_inputs, dim3(blocks(rows * k, 256)), dim3(256), 0, s, x, u, en, B, n, w, z);
  hipError_t e = gemm<float, uint16_t, false, true>(z, k, w1, k, a, h, (int)rows, h, k, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias_tanh, dim3(blocks(rows * h, 256)), dim3(256), 0, s, a, b1, rows, h);
  e = gemm<float, uint16_t, false, false>(a, h, w2, 1, y, 1, (int)rows, 1, h, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_bias1, dim3(blocks(rows, 256)), dim3(256), 0, s, y, b2, rows);
  return hipGetLastError();
}

constexpr int kMseBlocks = 256;

// loss (device double at loss_out[idx]) and gradient (FP32, packed layout).
hipError_t mixer_loss_grad(const uint16_t* p16, int w, int h, const float* u, const float* en, int n, const float* x,
                           const float* t, int B, float* scratch, double* part, float* grad, double* loss_out,
                           int idx, hipStream_t s) {
  const int k = mixer_features(w);
  const size_t rows = (size_t)B * n;
  float* z = scratch;
  float* a = z + rows * k;
  float* y = a + rows * h;
  float* da = y + rows;
  float* split = da + rows * h;
  hipError_t e = mixer_forward(p16, w, h, u, en, n, x, B, y, scratch, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mse, dim3(kMseBlocks), dim3(256), 0, s, y, t, rows, part);   // y := dY
  hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, part, kMseBlocks, 1.0 / (double)rows, loss_out, idx);
  const uint16_t* w2 = p16 + (size_t)h * k + h;
  float* gw1 = grad;
  float* gb1 = gw1 + (size_t)h * k;
  float* gw2 = gb1 + h;
  float* gb2 = gw2 + h;
  // gw2 (h) = A^T dY ; gb2 = sum dY
  e = gemm_splitk<float, float, true, false>(a, h, y, 1, gw2, h, 1, (int)rows, split, s);
  if (e != hipSuccess) return e;
  e = colsum(y, rows, 1, gb2, split, s);
  if (e != hipSuccess) return e;
  // dA (rows x h) = dY w2^T (outer product), then dZ = dA (1 - A^2)
  e = gemm<float, uint16_t, false, false>(y, 1, w2, h, da, h, (int)rows, h, 1, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_tanh_back, dim3(blocks(rows * h, 256)), dim3(256), 0, s, da, a, rows * h);
  // gW1 (h x k) = dZ^T Z ; gb1 = colsum(dZ)
  e = gemm_splitk<float, float, true, false>(da, h, z, k, gw1, h, k, (int)rows, split, s);
  if (e != hipSuccess) return e;
  e = colsum(da, rows, h, gb1, split, s);
  if (e != hipSuccess) return e;
  return hipGetLastError();
}

hipError_t mixer_adam(float* p, uint16_t* p16, float* m, float* v, const float* g, size_t count, float lr,
                      int step, hipStream_t s) {
  const double beta1 = 0.9, beta2 = 0.999;
  const float c1 = (float)(1.0 / (1.0 - std::pow(beta1, step)));
  const float c2 = (float)(1.0 / (1.0 - std::pow(beta2, step)));
  hipLaunchKernelGGL(k_adam, dim3(blocks(count, 256)), dim3(256), 0, s, p, p16, m, v, g, count, lr, (float)beta1,
                     (float)beta2, 1e-8f, c1, c2);
  return hipGetLastError();
}

hipError_t mixer_init(float* p, uint16_t* p16, int w, int h, uint64_t seed, hipStream_t s) {
  hipLaunchKernelGGL(k_init_params, dim3(blocks(mixer_param_count(w, h), 256)), dim3(256), 0, s, p, p16,
                     mixer_features(w), h, seed);
  return hipGetLastError();
}

// ---------------------------------------------------------------- SCF vectors

namespace {

// out[i] = c[i * ld + i]
__global__ void k_get_diag(const float* c, int n, size_t ld, double* out) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = c[(size_t)i * ld + i];
}

// W = diag(U_i s v_i) as a full n x n matrix (off-diagonal zeros written too).
__global__ void k_set_diag(float* w, int n, const float* u, const double* v, double s) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (size_t)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  w[e] = i == j ? (float)((double)u[i] * s * v[i]) : 0.0f;
}

// chi = s (a + b) (b may be null)
__global__ void k_combine(float* chi, const float* a, const float* b, double s, size_t n2) {
  const size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n2) chi[e] = (float)(s * ((double)a[e] + (b ? (double)b[e] : 0.0)));
}

// One 1024-thread block: out[q] = x_q . y_q for q < nq pairs of n-vectors (FP64).
__global__ __launch_bounds__(1024) void k_dots(const double* const* xs, const double* const* ys, int nq, int n,
                                               double* out) {
  __shared__ double red[16];
  for (int q = 0; q < nq; ++q) {
    double acc = 0.0;
    for (int i = threadIdx.x; i < n; i += 1024) acc += xs[q][i] * ys[q][i];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < 16; ++w) t += red[w];
      out[q] = t;
    }
    __syncthreads();
  }
}

// out = sum_q c_q x_q over nq vectors (coefficients on the device).
__global__ void k_lincomb(double* out, const double* const* xs, const double* c, int nq, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double acc = 0.0;
  for (int q = 0; q < nq; ++q) acc += c[q] * xs[q][i];
  out[i] = acc;
}

// x = (float)(r * inv)
__global__ void k_to_float(float* x, const double* r, double inv, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = (float)(r[i] * inv);
}

// out = v + alpha r + scale y  (y FP32, may be null)
__global__ void k_step_vec(double* out, const double* v, const double* r, double alpha, const float* y,
                           double scale, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) out[i] = v[i] + alpha * r[i] + (y ? scale * (double)y[i] : 0.0);
}

// r = f - v ; record (FP32 copies) when the pointers are set
__global__ void k_residual(double* r, const double* f, const double* v, int n, float* rec_v, float* rec_r) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  r[i] = f[i] - v[i];
  if (rec_v) rec_v[i] = (float)v[i];
  if (rec_r) rec_r[i] = (float)r[i];
}

// f = d_a + diag(cw) (cw may be null)
__global__ void k_fvec(double* f, const double* da, const float* cw, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) f[i] = da[i] + (cw ? (double)cw[(size_t)i * n + i] : 0.0);
}

// Training pairs of the learned mixer: for kept record row j = rows[b],
// x_b = sqrt(n) r_j / ||r_j||, t_b = sqrt(n) (v* - v_j - mix r_j) / ||r_j||
// (||r_j|| in FP64).  One workgroup per output row.
__global__ __launch_bounds__(256) void k_mixer_pairs(const float* v, const float* r, const float* vstar,
                                                     const int* rows, int n, float mix, float* x, float* t) {
  __shared__ double s_red[4];
  __shared__ double s_inv;
  const int j = rows[blockIdx.x];
  const float* rj = r + (size_t)j * n;
  const float* vj = v + (size_t)j * n;
  double acc = 0.0;
  for (int i = threadIdx.x; i < n; i += 256) acc += (double)rj[i] * (double)rj[i];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if ((threadIdx.x & 63) == 0) s_red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double nrm = sqrt((s_red[0] + s_red[1] + s_red[2] + s_red[3]) / (double)n);   // ||r|| / sqrt(n)
    s_inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  }
  __syncthreads();
  const float inv = (float)s_inv;
  float* xb = x + (size_t)blockIdx.x * n;
  float* tb = t + (size_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += 256) {
    xb[i] = rj[i] * inv;
    tb[i] = (vstar[i] - vj[i] - mix * rj[i]) * inv;
  }
}

// dst row b = src row perm[b] (rows of n floats).
__global__ __launch_bounds__(256) void k_gather_rows(const float* src, const int* perm, int n, float* dst) {
  const float* sr = src + (size_t)perm[blockIdx.x] * n;
  float* dr = dst + (size_t)blockIdx.x * n;
  for (int i = threadIdx.x; i < n; i += 256) dr[i] = sr[i];
}

}  // namespace

hipError_t mixer_pairs(const float* v, const float* r, const float* vstar, const int* rows, int nrows, int n,
                       float mix, float* x, float* t, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_mixer_pairs, dim3(nrows), dim3(256), 0, s, v, r, vstar, rows, n, mix, x, t);
  return hipGetLastError();
}

hipError_t mixer_gather_rows(const float* src, const int* perm, int nrows, int n, float* dst, hipStream_t s) {
  if (nrows <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_gather_rows, dim3(nrows), dim3(256), 0, s, src, perm, n, dst);
  return hipGetLastError();
}

hipError_t scf_get_diag(const float* c, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_get_diag, dim3(blocks(n, 256)), dim3(256), 0, s, c, n, (size_t)n, out);
  return hipGetLastError();
}
hipError_t scf_set_diag(float* w, int n, const float* u, const double* v, double spin, hipStream_t s) {
  hipLaunchKernelGGL(k_set_diag, dim3(blocks((size_t)n * n, 256)), dim3(256), 0, s, w, n, u, v, spin);
  return hipGetLastError();
}
hipError_t scf_combine(float* chi, const float* a, const float* b, double spin, size_t n2, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(blocks(n2, 256)), dim3(256), 0, s, chi, a, b, spin, n2);
  return hipGetLastError();
}
hipError_t scf_dots(const double* const* xs, const double* const* ys, int nq, int n, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_dots, dim3(1), dim3(1024), 0, s, xs, ys, nq, n, out);
  return hipGetLastError();
}
hipError_t scf_lincomb(double* out, const double* const* xs, const double* c, int nq, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_lincomb, dim3(blocks(n, 256)), dim3(256), 0, s, out, xs, c, nq, n);
  return hipGetLastError();
}
hipError_t scf_to_float(float* x, const double* r, double inv, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_to_float, dim3(blocks(n, 256)), dim3(256), 0, s, x, r, inv, n);
  return hipGetLastError();
}
hipError_t scf_step(double* out, const double* v, const double* r, double alpha, const float* y, double scale,
                    int n, hipStream_t s) {
  hipLaunchKernelGGL(k_step_vec, dim3(blocks(n, 256)), dim3(256), 0, s, out, v, r, alpha, y, scale, n);
  return hipGetLastError();
}
hipError_t scf_residual(double* r, const double* f, const double* v, int n, float* rec_v, float* rec_r,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_residual, dim3(blocks(n, 256)), dim3(256), 0, s, r, f, v, n, rec_v, rec_r);
  return hipGetLastError();
}
hipError_t scf_fvec(double* f, const double* da, const float* cw, int n, hipStream_t s) {
  hipLaunchKernelGGL(k_fvec, dim3(blocks(n, 256)), dim3(256), 0, s, f, da, cw, n);
  return hipGetLastError();
}

}  // namespace dmpt
