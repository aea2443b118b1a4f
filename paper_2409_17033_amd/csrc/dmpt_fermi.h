// Internal launchers of the finite-temperature path (dmpt_fermi.hip).  All
// matrices are n_pad x n_pad row-major FP32 (zero padded beyond n).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace dmpt {

// dst = scale (sym(src) - shift I_n), sym(S) = (S + S^T) / 2, src n x n (ld n).
hipError_t launch_fermi_start(const float* src, int n, int n_pad, double scale, double shift, float* dst,
                              hipStream_t s);
// z = a x + b y + d I_nd (y may be NULL; I_nd: ones on the first nd diagonal entries).
hipError_t launch_axpby(float* z, const float* x, float a, const float* y, float b, float d, int nd, int n_pad,
                        hipStream_t s);
// out = alpha (in + in^T) + beta x (x may be NULL); out must not alias in.
hipError_t launch_symm(const float* in, float alpha, const float* x, float beta, float* out, int n_pad,
                       hipStream_t s);
// FP64 per-row-block partials over the leading n x n block: part[2b] = trace,
// part[2b + 1] = sum of squares, b = 0 .. n_pad / 4 - 1 (four rows per block).
hipError_t launch_trace_sq(const float* m, int n, int n_pad, double* part, hipStream_t s);
int trace_sq_blocks(int n_pad);

}  // namespace dmpt
