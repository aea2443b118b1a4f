// Internal launchers of the self-consistent loop and its learned mixer
// (dmpt_mixer.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace dmpt {

// Learned mixer: site-local network with window w, hidden width h; site
// input [x window | on-site energy window | U_i] (k = 4w + 3 features);
// parameter layout [W1 (h x k) | b1 | w2 | b2].
inline int mixer_features(int w) { return 4 * w + 3; }
size_t mixer_param_count(int w, int h);
size_t mixer_scratch_floats(int n, int w, int h, int B);
hipError_t mixer_init(float* p, uint16_t* p16, int w, int h, uint64_t seed, hipStream_t s);
hipError_t mixer_forward(const uint16_t* p16, int w, int h, const float* u, const float* e, int n, const float* x,
                         int B, float* y, float* scratch, hipStream_t s);
hipError_t mixer_loss_grad(const uint16_t* p16, int w, int h, const float* u, const float* e, int n, const float* x,
                           const float* t, int B, float* scratch, double* part, float* grad, double* loss_out,
                           int idx, hipStream_t s);
// diag(M) of an n x n row-major matrix as FP32 (the on-site energies of H0).
hipError_t mixer_diag(const float* m, int n, float* out, hipStream_t s);
// Mixer training pairs from recorded rows rows[0..nrows) of (v, r), and a
// row gather dst[b] = src[perm[b]].
hipError_t mixer_pairs(const float* v, const float* r, const float* vstar, const int* rows, int nrows, int n,
                       float mix, float* x, float* t, hipStream_t s);
hipError_t mixer_gather_rows(const float* src, const int* perm, int nrows, int n, float* dst, hipStream_t s);
hipError_t mixer_adam(float* p, uint16_t* p16, float* m, float* v, const float* g, size_t count, float lr,
                      int step, hipStream_t s);

// Self-consistent loop vectors (dmpt_mixer.hip); state vectors are FP64, n-long.
hipError_t scf_get_diag(const float* c, int n, double* out, hipStream_t s);
hipError_t scf_set_diag(float* w, int n, const float* u, const double* v, double spin, hipStream_t s);
hipError_t scf_combine(float* chi, const float* a, const float* b, double spin, size_t n2, hipStream_t s);
hipError_t scf_dots(const double* const* xs, const double* const* ys, int nq, int n, double* out, hipStream_t s);
hipError_t scf_lincomb(double* out, const double* const* xs, const double* c, int nq, int n, hipStream_t s);
hipError_t scf_to_float(float* x, const double* r, double inv, int n, hipStream_t s);
hipError_t scf_step(double* out, const double* v, const double* r, double alpha, const float* y, double scale,
                    int n, hipStream_t s);
hipError_t scf_residual(double* r, const double* f, const double* v, int n, float* rec_v, float* rec_r,
                        hipStream_t s);
hipError_t scf_fvec(double* f, const double* da, const float* cw, int n, hipStream_t s);

}  // namespace dmpt
